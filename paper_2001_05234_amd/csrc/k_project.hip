// k_project.hip -- the projection step around the solve (the pressure correction that follows
// eq. (up)): the divergence fused into the forward x transform, and the correction kernel.
#include "kcommon.h"

namespace cans {


// ---------------------------------------------------------------------------
// Projection step (the pressure correction that follows eq. (up)):
//   f = D u / gdt  ->  Phi = L_h^{-1} f  ->  u -= gdt G Phi,  p += Phi.
// Staggered velocity: u on the +x face of each cell, v on the +y face, w on
// the +z face; every axis periodic (the face below the first cell wraps) or
// bounded by walls (zero normal velocity below the first cell; the last face
// is the wall and keeps its value, the gradient there being zero).
struct DivArgs {
    const double *u, *v, *w;
    const double *dzf;
    int nx, ny, nz;
    int px, py, pz;             // periodic axes
    double idx, idy, igdt;      // 1/dx, 1/dy, 1/gdt
};

// D u / gdt at the cell centres, fused into the forward x transform (FP64):
// each point's divergence is formed where the transform reads its input.
template <int KIND>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(4)))
void k_div_xfwd(double *out, long nlines, XGeom g, const cx<double> *__restrict__ tw, DivArgs d)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const Tile<AX_X, double> tile{reinterpret_cast<cx<double> *>(smem), g.L, g.RS, g.psh};
    const int n = g.n, ny = d.ny;
    const long line0 = (long)blockIdx.x * g.L;
    const int k0 = (int)(line0 / ny), j0 = (int)(line0 - (long)k0 * ny);
    const size_t plane = (size_t)n * ny;
    auto put = [&](int q, int l, double v) {
        const long line = line0 + l;
        if (line < nlines) out[(size_t)line * n + q] = v;
    };
    auto src = [&](int e, int l) -> double {
        const long line = line0 + l;
        if (line >= nlines) return 0.0;
        const int k = line_level(line, line0, k0, j0, ny), j = (int)(line - (long)k * ny);
        const size_t gi = (size_t)line * n + e;
        const double uw = e > 0 ? d.u[gi - 1] : (d.px ? d.u[gi + n - 1] : 0.0);
        const double vs = j > 0 ? d.v[gi - n] : (d.py ? d.v[gi + (size_t)(ny - 1) * n] : 0.0);
        const double wb = k > 0 ? d.w[gi - plane] : (d.pz ? d.w[gi + (size_t)(d.nz - 1) * plane] : 0.0);
        return ((d.u[gi] - uw) * d.idx + (d.v[gi] - vs) * d.idy + (d.w[gi] - wb) / d.dzf[k]) * d.igdt;
    };
    tile_transform<KIND, true, AX_X, true, false>(threadIdx.x, kThreads, g, src, put, tile, tile, tw, BlockSync());
}

struct CorrArgs {
    double *u, *v, *w, *p;
    const double *phi;
    const double *zgc;          // 1/dzc_k across the +z face of level k (0 on a wall face)
    int nx, ny, nz;
    int px, py, pz;
    double gdx, gdy, gdt;       // gdt/dx, gdt/dy, gdt
    double alpha;               // implicit diffusion: p += Phi - alpha L_h Phi
    LapArgs la;                 // L_h of Phi (the pressure's ghost rules)
};

// u -= gdt G Phi on the +faces and p += Phi (LAP: p += Phi - alpha L_h Phi,
// the pressure update of implicit diffusion); one block per x line.
template <bool LAP>
__global__ __launch_bounds__(256) void k_project_correct(CorrArgs c)
{
    const int line = (int)blockIdx.x;
    const int k = line / c.ny, j = line - k * c.ny;
    const size_t plane = (size_t)c.nx * c.ny, base = (size_t)line * c.nx;
    const double gz = c.gdt * c.zgc[k];
    for (int i = threadIdx.x; i < c.nx; i += 256) {
        const size_t e = base + i;
        const double f0 = c.phi[e];
        const double fe = i < c.nx - 1 ? c.phi[e + 1] : (c.px ? c.phi[e - (c.nx - 1)] : f0);
        const double fn = j < c.ny - 1 ? c.phi[e + c.nx] : (c.py ? c.phi[e - (size_t)(c.ny - 1) * c.nx] : f0);
        const double ft = k < c.nz - 1 ? c.phi[e + plane] : (c.pz ? c.phi[e - (size_t)(c.nz - 1) * plane] : f0);
        c.u[e] -= c.gdx * (fe - f0);
        c.v[e] -= c.gdy * (fn - f0);
        c.w[e] -= gz * (ft - f0);
        if constexpr (LAP) c.p[e] += f0 - c.alpha * lap_point(c.phi, i, j, k, c.la);
        else c.p[e] += f0;
    }
}

// ---------------------------------------------------------------------------
// Time-step bound of eq. (dt) on the staggered velocity, its advective part
// as the Listing of Section 3 evaluates it: at the +x, +y, +z face of each
// cell, the face-normal component plus the magnitudes of the four-point
// means of the two others, each over its spacing (dx, dy, dzf_k; the centre
// distance dzc_k at z faces).  Out-of-range neighbours: a component one face
// below the first cell along its own axis wraps or is zero at a wall; one
// cell beyond the last along another axis wraps or is the no-slip mirror
// (negated last value).
struct RateArgs {
    const double *u, *v, *w;
    const double *dzf;          // cell widths
    const double *dzc;          // centre distance across the +z face of each level (mirror cell at a wall)
    int nx, ny, nz;
    int per[3];                 // periodic x, y, z
    double idx, idy;
};

// component `comp` (0 u, 1 v, 2 w) at cell (i, j, k), indices one past
// either end allowed as described above
static __device__ inline double vel_at(const RateArgs &r, int comp, int i, int j, int k)
{
    const double *f = comp == 0 ? r.u : (comp == 1 ? r.v : r.w);
    int idx[3] = {i, j, k};
    const int n[3] = {r.nx, r.ny, r.nz};
    double sgn = 1.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (idx[a] < 0) {           // below the first cell: only along the component's own axis
            if (!r.per[a]) return 0.0;
            idx[a] = n[a] - 1;
        } else if (idx[a] >= n[a]) {  // beyond the last cell: only across
            if (r.per[a]) {
                idx[a] = 0;
            } else {
                idx[a] = n[a] - 1;
                sgn = -sgn;
            }
        }
    }
    return sgn * f[(size_t)idx[0] + (size_t)r.nx * ((size_t)idx[1] + (size_t)r.ny * idx[2])];
}

// an interior cell (every neighbour the rates use exists): the same loads and
// arithmetic as below by direct offsets
static __device__ inline double cell_rate_interior(const RateArgs &r, size_t e, int k)
{
    const size_t sy = (size_t)r.nx, sz = (size_t)r.nx * r.ny;
    const double *u = r.u + e, *v = r.v + e, *w = r.w + e;
    const double idz = 1.0 / r.dzf[k];
    const double ux = fabs(u[0]);
    const double vx = 0.25 * fabs(v[0] + v[-(ptrdiff_t)sy] + v[1] + v[1 - (ptrdiff_t)sy]);
    const double wx = 0.25 * fabs(w[0] + w[-(ptrdiff_t)sz] + w[1] + w[1 - (ptrdiff_t)sz]);
    const double rx = ux * r.idx + vx * r.idy + wx * idz;
    const double uy = 0.25 * fabs(u[0] + u[-1] + u[sy] + u[sy - 1]);
    const double vy = fabs(v[0]);
    const double wy = 0.25 * fabs(w[0] + w[-(ptrdiff_t)sz] + w[sy] + w[(ptrdiff_t)sy - (ptrdiff_t)sz]);
    const double ry = uy * r.idx + vy * r.idy + wy * idz;
    const double uz = 0.25 * fabs(u[0] + u[-1] + u[sz] + u[sz - 1]);
    const double vz = 0.25 * fabs(v[0] + v[-(ptrdiff_t)sy] + v[sz] + v[sz - sy]);
    const double wz = fabs(w[0]);
    const double rz = uz * r.idx + vz * r.idy + wz / r.dzc[k];
    return fmax(rx, fmax(ry, rz));
}

static __device__ inline double cell_rate(const RateArgs &r, int i, int j, int k)
{
    if (i > 0 && i < r.nx - 1 && j > 0 && j < r.ny - 1 && k > 0 && k < r.nz - 1)
        return cell_rate_interior(r, (size_t)i + (size_t)r.nx * ((size_t)j + (size_t)r.ny * k), k);
    const double idz = 1.0 / r.dzf[k];
    const double ux = fabs(vel_at(r, 0, i, j, k));
    const double vx = 0.25 * fabs(vel_at(r, 1, i, j, k) + vel_at(r, 1, i, j - 1, k) + vel_at(r, 1, i + 1, j, k) +
                                  vel_at(r, 1, i + 1, j - 1, k));
    const double wx = 0.25 * fabs(vel_at(r, 2, i, j, k) + vel_at(r, 2, i, j, k - 1) + vel_at(r, 2, i + 1, j, k) +
                                  vel_at(r, 2, i + 1, j, k - 1));
    const double rx = ux * r.idx + vx * r.idy + wx * idz;
    const double uy = 0.25 * fabs(vel_at(r, 0, i, j, k) + vel_at(r, 0, i - 1, j, k) + vel_at(r, 0, i, j + 1, k) +
                                  vel_at(r, 0, i - 1, j + 1, k));
    const double vy = fabs(vel_at(r, 1, i, j, k));
    const double wy = 0.25 * fabs(vel_at(r, 2, i, j, k) + vel_at(r, 2, i, j, k - 1) + vel_at(r, 2, i, j + 1, k) +
                                  vel_at(r, 2, i, j + 1, k - 1));
    const double ry = uy * r.idx + vy * r.idy + wy * idz;
    const double uz = 0.25 * fabs(vel_at(r, 0, i, j, k) + vel_at(r, 0, i - 1, j, k) + vel_at(r, 0, i, j, k + 1) +
                                  vel_at(r, 0, i - 1, j, k + 1));
    const double vz = 0.25 * fabs(vel_at(r, 1, i, j, k) + vel_at(r, 1, i, j - 1, k) + vel_at(r, 1, i, j, k + 1) +
                                  vel_at(r, 1, i, j - 1, k + 1));
    const double wz = fabs(vel_at(r, 2, i, j, k));
    const double rz = uz * r.idx + vz * r.idy + wz / r.dzc[k];
    return fmax(rx, fmax(ry, rz));
}

constexpr int kRateBlocks = 2048;

// block maxima of the face rates over lines b, b + grid, ... (x lines j + ny k)
__global__ __launch_bounds__(256) void k_dt_rates(RateArgs r, double *__restrict__ part)
{
    const int nlines = r.ny * r.nz;
    double m = 0.0;
    for (int line = blockIdx.x; line < nlines; line += gridDim.x) {
        const int k = line / r.ny, j = line - k * r.ny;
        for (int i = threadIdx.x; i < r.nx; i += 256) m = fmax(m, cell_rate(r, i, j, k));
    }
    double z = 0.0;
    block_max2(m, z);
    if (threadIdx.x == 0) part[blockIdx.x] = m;
}

// dt = min(sqrt(3) / max rate, 1.65 dl^2 / nu): the largest block maximum
// (a maximum is exact in any order); +inf for a field at rest without nu
__global__ __launch_bounds__(256) void k_dt_final(const double *__restrict__ part, int nblk, double visc_bound,
                                                  double *__restrict__ dt)
{
    double m = 0.0, z = 0.0;
    for (int b = threadIdx.x; b < nblk; b += 256) m = fmax(m, part[b]);
    block_max2(m, z);
    if (threadIdx.x == 0) {
        const double adv = m > 0.0 ? sqrt(3.0) / m : __builtin_inf();
        dt[0] = fmin(adv, visc_bound);
    }
}

int launch_div_xfwd(const Problem &pb, const double *u, const double *v, const double *w, double gdt, double *out,
                    hipStream_t s)
{
    const XGeom &g = pb.ax.gx64[1];
    const long nlines = (long)pb.ny * pb.nz;
    const dim3 grid((unsigned)((nlines + g.L - 1) / g.L));
    const size_t sh = tile_lds(AX_X, g, sizeof(double));
    DivArgs d{u, v, w, pb.d_dzf, pb.nx, pb.ny, pb.nz,
              pb.bc[0] == CANS_BC_PERIODIC, pb.bc[2] == CANS_BC_PERIODIC, pb.bc[4] == CANS_BC_PERIODIC,
              1.0 / pb.ax.h, 1.0 / pb.ay.h, 1.0 / gdt};
    // the projection step takes periodic or wall (Neumann) pressure boundaries
    if (pb.ax.kind == K_P)
        hipLaunchKernelGGL(k_div_xfwd<K_P>, grid, dim3(kThreads), sh, s, out, nlines, g, pb.ax.d_tw64, d);
    else if (pb.ax.kind == K_NN)
        hipLaunchKernelGGL(k_div_xfwd<K_NN>, grid, dim3(kThreads), sh, s, out, nlines, g, pb.ax.d_tw64, d);
    else
        return CANS_ERR_UNSUPPORTED;
    return check_launch();
}

int launch_project_correct(const Problem &pb, double *u, double *v, double *w, double *p, const double *phi,
                           double gdt, double alpha, hipStream_t s)
{
    CorrArgs c{u, v, w, p, phi, pb.d_zgc, pb.nx, pb.ny, pb.nz,
               pb.bc[0] == CANS_BC_PERIODIC, pb.bc[2] == CANS_BC_PERIODIC, pb.bc[4] == CANS_BC_PERIODIC,
               gdt / pb.ax.h, gdt / pb.ay.h, gdt, alpha, lapargs(pb)};
    if (alpha != 0.0)
        hipLaunchKernelGGL(k_project_correct<true>, dim3((unsigned)(pb.ny * pb.nz)), dim3(256), 0, s, c);
    else
        hipLaunchKernelGGL(k_project_correct<false>, dim3((unsigned)(pb.ny * pb.nz)), dim3(256), 0, s, c);
    return check_launch();
}

int dt_blocks(const Problem &pb)
{
    const long nlines = (long)pb.ny * pb.nz;
    return (int)(nlines < kRateBlocks ? nlines : kRateBlocks);
}

int launch_max_dt(const Problem &pb, const double *u, const double *v, const double *w, double nu, double *dt,
                  hipStream_t s)
{
    RateArgs r{u, v, w, pb.d_dzf, pb.d_dzc, pb.nx, pb.ny, pb.nz,
               {pb.bc[0] == CANS_BC_PERIODIC, pb.bc[2] == CANS_BC_PERIODIC, pb.bc[4] == CANS_BC_PERIODIC},
               1.0 / pb.ax.h, 1.0 / pb.ay.h};
    double dl = pb.ax.h < pb.ay.h ? pb.ax.h : pb.ay.h;
    for (double d : pb.dzf) dl = d < dl ? d : dl;
    const double visc = nu > 0.0 ? 1.65 * dl * dl / nu : __builtin_inf();
    const int nb = dt_blocks(pb);
    hipLaunchKernelGGL(k_dt_rates, dim3((unsigned)nb), dim3(256), 0, s, r, pb.dt_part);
    hipLaunchKernelGGL(k_dt_final, dim3(1), dim3(256), 0, s, pb.dt_part, nb, visc, dt);
    return check_launch();
}
}  // namespace cans

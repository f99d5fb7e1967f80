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
};

// u -= gdt G Phi on the +faces and p += Phi; one block per x line.
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
        c.p[e] += f0;
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
    CANS_KIND_SWITCH(pb.ax.kind,
        hipLaunchKernelGGL(k_div_xfwd<KD>, grid, dim3(kThreads), sh, s, out, nlines, g, pb.ax.d_tw64, d));
    return check_launch();
}

int launch_project_correct(const Problem &pb, double *u, double *v, double *w, double *p, const double *phi,
                           double gdt, hipStream_t s)
{
    CorrArgs c{u, v, w, p, phi, pb.d_zgc, pb.nx, pb.ny, pb.nz,
               pb.bc[0] == CANS_BC_PERIODIC, pb.bc[2] == CANS_BC_PERIODIC, pb.bc[4] == CANS_BC_PERIODIC,
               gdt / pb.ax.h, gdt / pb.ay.h, gdt};
    hipLaunchKernelGGL(k_project_correct, dim3((unsigned)(pb.ny * pb.nz)), dim3(256), 0, s, c);
    return check_launch();
}
}  // namespace cans

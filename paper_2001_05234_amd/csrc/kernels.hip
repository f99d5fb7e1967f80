// kernels.hip -- gfx950 kernels of the direct Poisson solver (Section 2,
// eqs. (poi) and (poi_reduced)): LDS-tiled real-to-real transforms along x
// (contiguous lines) and y (tiles of adjacent x columns, coalesced rows, no
// global transpose), the FP64 column-wise tridiagonal solve along z (one lane
// per column, adjacent columns in adjacent lanes), and the FP64 residual /
// norm kernels of iterative refinement.
#include <hip/hip_runtime.h>

#include "cans_internal.h"
#include "dense_core.h"

namespace cans {

struct BlockSync {
    __device__ void operator()() const { __syncthreads(); }
};

#define CANS_KIND_SWITCH(kind, ...)                                  \
    switch (kind) {                                                  \
    case K_P: { constexpr int KD = K_P; __VA_ARGS__; } break;        \
    case K_NN: { constexpr int KD = K_NN; __VA_ARGS__; } break;      \
    case K_DD: { constexpr int KD = K_DD; __VA_ARGS__; } break;      \
    case K_ND: { constexpr int KD = K_ND; __VA_ARGS__; } break;      \
    default: { constexpr int KD = K_DN; __VA_ARGS__; } break;        \
    }

static int check_launch()
{
    return hipGetLastError() == hipSuccess ? CANS_OK : CANS_ERR_HIP;
}

// ---------------------------------------------------------------------------
// Deterministic block sum of three doubles (fixed order): result in lane 0.
__device__ void block_sum3(double &a, double &b, double &c)
{
    __shared__ double red[3][kThreads / 64];
    for (int off = 32; off > 0; off >>= 1) {
        a += __shfl_down(a, off, 64);
        b += __shfl_down(b, off, 64);
        c += __shfl_down(c, off, 64);
    }
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) { red[0][w] = a; red[1][w] = b; red[2][w] = c; }
    __syncthreads();
    if (threadIdx.x == 0) {
        a = 0; b = 0; c = 0;
        for (int i = 0; i < kThreads / 64; ++i) { a += red[0][i]; b += red[1][i]; c += red[2][i]; }
    }
    __syncthreads();
}

// block maxima of two non-negative values (exact in any order)
__device__ void block_max2(double &a, double &b)
{
    __shared__ double red[2][kThreads / 64];
    for (int off = 32; off > 0; off >>= 1) {
        a = fmax(a, __shfl_down(a, off, 64));
        b = fmax(b, __shfl_down(b, off, 64));
    }
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) { red[0][w] = a; red[1][w] = b; }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 0; i < kThreads / 64; ++i) { a = fmax(a, red[0][i]); b = fmax(b, red[1][i]); }
    }
    __syncthreads();
}

// one block partial of the residual passes (thread 0 writes)
__device__ void put_partial(double *partials, unsigned b, double srr, double sff, double spw, double rmax,
                            double fmax_)
{
    block_sum3(srr, sff, spw);
    block_max2(rmax, fmax_);
    if (threadIdx.x == 0) {
        double *q = partials + (size_t)kNP * b;
        q[0] = srr;
        q[1] = sff;
        q[2] = spw;
        q[3] = rmax;
        q[4] = fmax_;
    }
}

// ---------------------------------------------------------------------------
// Blocks are dispatched round-robin over the 8 XCDs; remap so that each XCD
// runs a contiguous range of tiles (neighbouring y tiles share cache lines).
__device__ inline unsigned xcd_remap(unsigned b, unsigned nblk)
{
    const unsigned q = nblk / 8, r = nblk % 8, x = b % 8, i = b / 8;
    return x < r ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

// z level of line `line` (rows j + ny*k) inside a tile starting at line0
__device__ inline int line_level(long line, long line0, int k0, int j0, int ny)
{
    const long d = line - line0;
    return (j0 + d < ny) ? k0 : (int)(line / ny);
}

// x transform: a block holds L consecutive x lines (rows j + ny*k).
// EPI 0: out = v;  EPI 1: out = out + v - info[I_MEANP] (refinement update).
// `wsum_part` (optional, forward only): block partial sums of dzf_k * in in
// FP64, so the exact weighted mean of the rhs is known in refinement mode.
// At least 4 waves per SIMD: the staged FP64 inverses would otherwise take
// 145 VGPRs and run 3 (the cap costs them a small spill and is faster).
template <int KIND, bool FWD, typename T, typename Tin, typename Tout, int EPI>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(4)))
void k_xform_x(const Tin *in, Tout *out, long nlines, XGeom g,
                                                      const cx<T> *__restrict__ tw,
                                                      const double *__restrict__ info,
                                                      const int *__restrict__ done,
                                                      const double *__restrict__ dzf, int ny,
                                                      double *__restrict__ wsum_part)
{
    if (done && *done) return;
    extern __shared__ __align__(16) unsigned char smem[];
    const Tile<AX_X, T> tile{reinterpret_cast<cx<T> *>(smem), g.L, g.RS, g.psh};
    const int n = g.n;
    const long line0 = (long)blockIdx.x * g.L;
    const int k0 = (int)(line0 / ny), j0 = (int)(line0 - (long)k0 * ny);
    const double mp = EPI == 1 ? info[I_MEANP] : 0.0;
    auto put = [&](int q, int l, T v) {
        const long line = line0 + l;
        if (line < nlines) {
            const size_t idx = (size_t)line * n + q;
            if (EPI == 1) out[idx] = (Tout)((double)out[idx] + (double)v - mp);
            else out[idx] = (Tout)v;
        }
    };
    // inverse real-DFT / DCT / DST synthesis reads every input twice: stage
    // the lines in LDS with coalesced loads first
    constexpr bool STAGED = !FWD && (KIND == K_P || KIND == K_NN || KIND == K_DD);
    if constexpr (STAGED) {
        for (int idx = threadIdx.x; idx < n * g.L; idx += kThreads) {
            const int l = (int)udiv((unsigned)idx, (unsigned)n, g.magN), e = idx - l * n;
            const long line = line0 + l;
            tile_real(tile, e, l) = line < nlines ? (T)in[line * n + e] : T(0);
        }
        __syncthreads();
        auto src = [&](int e, int l) -> T { return tile_real(tile, e, l); };
        tile_transform<KIND, FWD, AX_X, true, true>(threadIdx.x, kThreads, g, src, put, tile, tile, tw, BlockSync());
    } else {
        double acc = 0;
        auto src = [&](int e, int l) -> T {
            const long line = line0 + l;
            if (line >= nlines) return T(0);
            const Tin x = in[line * n + e];
            if (wsum_part) acc += dzf[line_level(line, line0, k0, j0, ny)] * (double)x;
            return (T)x;
        };
        tile_transform<KIND, FWD, AX_X, true, false>(threadIdx.x, kThreads, g, src, put, tile, tile, tw,
                                                     BlockSync());
        if (wsum_part) {
            double z1 = 0, z2 = 0;
            block_sum3(acc, z1, z2);
            if (threadIdx.x == 0) {
                wsum_part[kNP * blockIdx.x] = acc;
            }
        }
    }
}

// y transform: tile (t, k) holds columns i0 .. i0+L-1 of plane k, all ny
// rows; each global row segment of L elements is contiguous.
template <int KIND, bool FWD, typename T, typename Tio>
__global__ __launch_bounds__(kThreads) void k_xform_y(const Tio *in, Tio *out, int nx, int ny, int ntx, XGeom g,
                                                      const cx<T> *__restrict__ tw,
                                                      const int *__restrict__ done)
{
    if (done && *done) return;
    extern __shared__ __align__(16) unsigned char smem[];
    const Tile<AX_Y, T> tile{reinterpret_cast<cx<T> *>(smem), g.L, g.RS, g.psh};
    const unsigned t = xcd_remap(blockIdx.x, gridDim.x);
    const int i0 = (int)(t % ntx) * g.L;
    const size_t base = (size_t)(t / ntx) * nx * ny;
    auto put = [&](int q, int l, T v) {
        const int i = i0 + l;
        if (i < nx) out[base + (size_t)q * nx + i] = (Tio)v;
    };
    // y tiles read their rows directly (staging through LDS measured slower)
    constexpr bool STAGED = false;
    if constexpr (STAGED) {
        for (int idx = threadIdx.x; idx < ny * g.L; idx += kThreads) {
            const int l = idx & (g.L - 1), e = idx >> g.lgL, i = i0 + l;
            tile_real(tile, e, l) = i < nx ? (T)in[base + (size_t)e * nx + i] : T(0);
        }
        __syncthreads();
        auto src = [&](int e, int l) -> T { return tile_real(tile, e, l); };
        tile_transform<KIND, FWD, AX_Y, true, true>(threadIdx.x, kThreads, g, src, put, tile, tile, tw, BlockSync());
    } else {
        auto src = [&](int e, int l) -> T {
            const int i = i0 + l;
            return i < nx ? (T)in[base + (size_t)e * nx + i] : T(0);
        };
        tile_transform<KIND, FWD, AX_Y, true, false>(threadIdx.x, kThreads, g, src, put, tile, tile, tw,
                                                     BlockSync());
    }
}

// Residual of the current p fused with the forward x transform of it:
//   r = (f - removed mean) - L_h p   (FP64), out = T_x r (FP32);
// block partials: sums of |r|^2, |f - mean|^2, dzf p; maxima of |r|, |f - mean|.
template <int KIND>
__global__ __launch_bounds__(kThreads) void k_resid_xfwd(const double *__restrict__ f,
                                                         const double *__restrict__ p, float *out,
                                                         long nlines, XGeom g,
                                                         const cx<float> *__restrict__ tw, LapArgs la,
                                                         const double *__restrict__ dzf,
                                                         const double *__restrict__ info,
                                                         double *__restrict__ partials,
                                                         const int *__restrict__ done)
{
    if (*done) return;
    extern __shared__ __align__(16) unsigned char smem[];
    const Tile<AX_X, float> tile{reinterpret_cast<cx<float> *>(smem), g.L, g.RS, g.psh};
    const int n = g.n, ny = la.ny;
    const long line0 = (long)blockIdx.x * g.L;
    const int k0 = (int)(line0 / ny), j0 = (int)(line0 - (long)k0 * ny);
    const double mf = info[I_REMOVED];
    double srr = 0, sff = 0, spw = 0, rmax = 0, fmx = 0;
    // residual of the tile's lines into LDS (coalesced, each point once)
    auto one = [&](int e, int l, long line, int j, int k) {
        const size_t gi = (size_t)line * n + e;
        const double fv = f[gi] - mf;
        const double r = fv - lap_point(p, e, j, k, la);
        srr += r * r;
        sff += fv * fv;
        rmax = fmax(rmax, fabs(r));
        fmx = fmax(fmx, fabs(fv));
        spw += dzf[k] * p[gi];
        tile_real(tile, e, l) = (float)r;
    };
    if (n % kThreads == 0) {
        // whole lines per thread group: line, j and k are uniform per pass
        for (int l = 0; l < g.L; ++l) {
            const long line = line0 + l;
            if (line < nlines) {
                const int k = line_level(line, line0, k0, j0, ny), j = (int)(line - (long)k * ny);
                for (int e = threadIdx.x; e < n; e += kThreads) one(e, l, line, j, k);
            } else {
                for (int e = threadIdx.x; e < n; e += kThreads) tile_real(tile, e, l) = 0.f;
            }
        }
    } else {
        for (int idx = threadIdx.x; idx < n * g.L; idx += kThreads) {
            const int l = (int)udiv((unsigned)idx, (unsigned)n, g.magN), e = idx - l * n;
            const long line = line0 + l;
            if (line < nlines) {
                const int k = line_level(line, line0, k0, j0, ny), j = (int)(line - (long)k * ny);
                one(e, l, line, j, k);
            } else {
                tile_real(tile, e, l) = 0.f;
            }
        }
    }
    __syncthreads();
    auto src = [&](int e, int l) -> float { return tile_real(tile, e, l); };
    auto put = [&](int q, int l, float v) {
        const long line = line0 + l;
        if (line < nlines) out[(size_t)line * n + q] = v;
    };
    tile_transform<KIND, true, AX_X, true, true>(threadIdx.x, kThreads, g, src, put, tile, tile, tw, BlockSync());
    put_partial(partials, blockIdx.x, srr, sff, spw, rmax, fmx);
}

// Residual norms only (the check after a correction): the same block
// partials as k_resid_xfwd over lines_per_block lines.
__global__ __launch_bounds__(kThreads) void k_resid_norm(const double *__restrict__ f,
                                                         const double *__restrict__ p, long nlines,
                                                         int lines_per_block, LapArgs la,
                                                         const double *__restrict__ dzf,
                                                         const double *__restrict__ info,
                                                         double *__restrict__ partials,
                                                         const int *__restrict__ done)
{
    if (*done) return;
    const int n = la.nx, ny = la.ny;
    const long line0 = (long)blockIdx.x * lines_per_block;
    const int k0 = (int)(line0 / ny), j0 = (int)(line0 - (long)k0 * ny);
    const double mf = info[I_REMOVED];
    double srr = 0, sff = 0, spw = 0, rmax = 0, fmx = 0;
    for (int l = 0; l < lines_per_block; ++l) {
        const long line = line0 + l;
        if (line >= nlines) break;
        const int k = line_level(line, line0, k0, j0, ny), j = (int)(line - (long)k * ny);
        const double wk = dzf[k];
        for (int e = threadIdx.x; e < n; e += kThreads) {
            const size_t gi = (size_t)line * n + e;
            const double fv = f[gi] - mf;
            const double r = fv - lap_point(p, e, j, k, la);
            srr += r * r;
            sff += fv * fv;
            rmax = fmax(rmax, fabs(r));
            fmx = fmax(fmx, fabs(fv));
            spw += wk * p[gi];
        }
    }
    put_partial(partials, blockIdx.x, srr, sff, spw, rmax, fmx);
}

// First level of the block-partial reductions: block b reduces its contiguous
// chunk of partials (fixed order) into sums[kNP b .. kNP b + kNP - 1].
constexpr int kReduceBlocks = 256;

__global__ __launch_bounds__(kThreads) void k_reduce1(const double *__restrict__ partials, int nblk,
                                                      double *__restrict__ sums, const int *__restrict__ done)
{
    if (done && *done) return;
    const int chunk = (nblk + kReduceBlocks - 1) / kReduceBlocks;
    const int lo = blockIdx.x * chunk, hi = min(nblk, lo + chunk);
    double a = 0, b = 0, c = 0, d = 0, e = 0;
    for (int i = lo + (int)threadIdx.x; i < hi; i += kThreads) {
        const double *q = partials + (size_t)kNP * i;
        a += q[0];
        b += q[1];
        c += q[2];
        d = fmax(d, q[3]);
        e = fmax(e, q[4]);
    }
    put_partial(sums, blockIdx.x, a, b, c, d, e);
}

// Sum the first-level sums in a fixed order, record the relative residual of
// check number `check` (2-norm, and the max norm beside it) and decide:
// converged (<= tol, 2-norm) or out of steps.
__global__ __launch_bounds__(kThreads) void k_finalize(const double *__restrict__ partials, int nblk,
                                                       int check, int max_iter, double tol,
                                                       double inv_wvol, int singular,
                                                       double *__restrict__ info, int *__restrict__ flag)
{
    if (flag[0]) return;
    double a = 0, b = 0, c = 0, d = 0, e = 0;
    for (int i = threadIdx.x; i < nblk; i += kThreads) {
        const double *q = partials + (size_t)kNP * i;
        a += q[0];
        b += q[1];
        c += q[2];
        d = fmax(d, q[3]);
        e = fmax(e, q[4]);
    }
    block_sum3(a, b, c);
    block_max2(d, e);
    if (threadIdx.x == 0) {
        const double rel = b > 0 ? sqrt(a / b) : sqrt(a);
        info[I_HIST + check] = rel;
        info[I_LAST] = rel;
        info[I_LINF] = e > 0 ? d / e : d;
        info[I_MEANP] = singular ? c * inv_wvol : 0.0;
        info[I_ITERS] = check;
        if (rel <= tol) {
            info[I_CONV] = 1;
            flag[0] = 1;
        } else if (check >= max_iter) {
            info[I_CONV] = 0;
            flag[0] = 1;
        }
    }
}

// Exact FP64 weighted mean of the rhs from the first pass's block sums:
// info[I_REMOVED] = sum dzf f / (nx ny sum dzf) when singular, else 0.
__global__ __launch_bounds__(kThreads) void k_mean_rhs(const double *__restrict__ partials, int nblk,
                                                       double inv_wvol, int singular,
                                                       double *__restrict__ info)
{
    double a = 0, b = 0, c = 0;
    for (int i = threadIdx.x; i < nblk; i += kThreads) a += partials[(size_t)kNP * i];
    block_sum3(a, b, c);
    if (threadIdx.x == 0) info[I_REMOVED] = singular ? a * inv_wvol : 0.0;
}

// Start-of-solve state, written by a kernel so the sequence can be captured.
__global__ void k_reset(double *__restrict__ info, int *__restrict__ flag)
{
    const int t = threadIdx.x;
    if (t < I_SIZE) info[t] = (t >= I_HIST || t == I_LAST) ? -1.0 : 0.0;
    if (t == 0) flag[0] = 0;
}

template <typename T>
__global__ __launch_bounds__(256) void k_zsolve(T *data, ZArgs a, const int *__restrict__ done)
{
    if (done && *done) return;
    const size_t col = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (col >= (size_t)a.nx * a.ny) return;
    zsolve_column(col, data, a);
}

static ZArgs zargs(const Problem &pb, double *removed);

// Partitioned column solve: CPB adjacent columns per block (64 or 32), z split
// into S segments of at most MMAX levels held in registers; a wave holds
// 64/CPB segments of the same columns (see zsolve_core.h).
template <typename T, int MMAX, int CPB, int NTMAX, bool FULL, bool CYC, bool PAD = false>
__global__ __launch_bounds__(NTMAX) void k_zsolve_part(T *data, ZArgs ag, const int *__restrict__ done)
{
    if (done && *done) return;
    constexpr int NQ = CYC ? 8 : 6;  // interface coefficients per segment
    __shared__ double coef[NQ * 1024];
    __shared__ double zabc[3 * 512];  // the z coefficients, staged once per block
    __shared__ double ends[CYC ? 4 * 64 : 1];  // CYC: first/last values per column
    constexpr int SPW = 64 / CPB;  // segments per wave
    // PAD: S * MMAX levels (<= 512 for every launched shape), padding rows
    // beyond nz
    const int nzp = PAD ? (int)(blockDim.x >> 6) * SPW * MMAX : ag.nz;
    for (int i = threadIdx.x; i < nzp; i += blockDim.x)
        zpad_row(ag, i, zabc[i], zabc[512 + i], zabc[1024 + i]);
    ZArgs a = ag;
    a.za = zabc;
    a.zb = zabc + 512;
    a.zc = zabc + 1024;
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
    const int c = lane % CPB, seg = w * SPW + lane / CPB;
    const int S = (int)(blockDim.x >> 6) * SPW;
    auto C = [&](int q, int s) -> double & { return coef[q * 1024 + s * CPB + c]; };
    const size_t col = (size_t)blockIdx.x * CPB + c;
    const ZSeg sg = zseg(nzp, S, seg);
    ZLane<MMAX, CYC> L;
    zp_load<MMAX, FULL, PAD>(L, data, a, col, sg);
    double out[NQ];
    zp_reduce<MMAX, FULL>(L, a, sg, out);
#pragma unroll
    for (int q = 0; q < NQ; ++q) C(q, seg) = out[q];
    __syncthreads();
    if (w == 0 && lane < CPB) {
        zp_interface<CYC>(
            S, [&](int s, int q) -> double & { return C(q, s); }, [&](int s) -> double & { return C(4, s); },
            [&](int s) -> double & { return C(5, s); }, [&](int s) -> double & { return C(6, s); },
            [&](int s) -> double & { return C(7, s); });
    }
    __syncthreads();
    const double xL = seg > 0 ? C(5, seg - 1) : 0.0;
    const double xR = seg < S - 1 ? C(4, seg + 1) : 0.0;
    if constexpr (CYC) {
        const double xL2 = seg > 0 ? C(7, seg - 1) : 0.0;
        const double xR2 = seg < S - 1 ? C(6, seg + 1) : 0.0;
        zp_finish<MMAX, FULL>(L, a, sg, xL, xR, xL2, xR2);
        // Sherman-Morrison: the column's first and last values of A'^-1 f and
        // A'^-1 u come from its first and last segment
        double y0, z0, yl, zl;
        zp_ends<MMAX, FULL>(L, sg, &y0, &z0, &yl, &zl);
        if (seg == 0) { ends[c] = y0; ends[64 + c] = z0; }
        if (seg == S - 1) { ends[128 + c] = yl; ends[192 + c] = zl; }
        __syncthreads();
        zp_sherman_morrison<MMAX, FULL>(L, a, sg, ends[c], ends[64 + c], ends[128 + c], ends[192 + c]);
    } else {
        zp_finish<MMAX, FULL>(L, a, sg, xL, xR);
    }
    zp_store<MMAX, FULL, PAD>(L, data, a, col, sg);
    if (a.singular && blockIdx.x == 0) {
        // the singular column, left out above: projected rhs, pinned last
        // row, zero weighted mean, by one thread with coef as workspace
        __syncthreads();
        if (threadIdx.x == 0) zsolve_singular_ws<T>(0, data, a, coef, coef + 512, 1);
    }
}

template <typename T>
static int launch_zsolve(const Problem &pb, T *data, double *removed, const int *done, hipStream_t s)
{
    const size_t plane = (size_t)pb.nx * pb.ny;
    const ZPart zp = zpart_shape(pb.nz, pb.cyclic != 0);
    ZArgs za = zargs(pb, removed);
    if (zp.mmax == 0) {
        hipLaunchKernelGGL(k_zsolve<T>, dim3((unsigned)((plane + 255) / 256)), dim3(256), 0, s, data, za, done);
        return check_launch();
    }
    const dim3 grid((unsigned)((plane + zp.cpb - 1) / zp.cpb)), block(zp.threads);
    const int S = (zp.threads / 64) * (64 / zp.cpb);
    const bool full = pb.nz == S * zp.mmax;  // every segment holds mmax levels
    // a FULL 16-level kernel keeps both segment sweeps unrolled in registers;
    // with at most 768 threads per block its register limit is 168, not 128
    const bool small = zp.threads <= 768;
#define CANS_ZP(MM, CPB, NT, FULLV, CYCV) \
    hipLaunchKernelGGL((k_zsolve_part<T, MM, CPB, NT, FULLV, CYCV>), grid, block, 0, s, data, za, done)
    if (pb.cyclic) {  // nz <= 128: 8-level segments of 64 columns
        if (full) CANS_ZP(8, 64, 1024, true, true); else CANS_ZP(8, 64, 1024, false, true);
        return check_launch();
    }
#undef CANS_ZP
    // non-periodic z always runs full segments: a ragged nz is padded to
    // S * mmax levels with decoupled rows (the level guards of a ragged
    // split cost ~15 % at nz = 383)
#define CANS_ZP(MM, CPB, NT, PADV) \
    hipLaunchKernelGGL((k_zsolve_part<T, MM, CPB, NT, true, false, PADV>), grid, block, 0, s, data, za, done)
#define CANS_ZP2(MM, CPB, NT) do { if (full) CANS_ZP(MM, CPB, NT, false); else CANS_ZP(MM, CPB, NT, true); } while (0)
    if (zp.mmax == 8) {
        CANS_ZP2(8, 64, 1024);
    } else if (zp.cpb == 64) {
        if (small) CANS_ZP2(16, 64, 768); else CANS_ZP2(16, 64, 1024);
    } else {
        if (small) CANS_ZP2(16, 32, 768); else CANS_ZP2(16, 32, 1024);
    }
#undef CANS_ZP2
#undef CANS_ZP
    return check_launch();
}

// ---------------------------------------------------------------------------
// Dense (matrix-core) x transforms of the refinement path: the same prologues
// and epilogues as the FFT kernels around dense_transform (32 lines a block).
template <bool FWD, typename Tin, typename Tout, int EPI>
__global__ __launch_bounds__(256) void k_dense_x(const Tin *in, Tout *out, long nlines, int n, unsigned magn,
                                                 const unsigned short *__restrict__ Wh,
                                                 const unsigned short *__restrict__ Wl,
                                                 const double *__restrict__ info, const int *__restrict__ done,
                                                 const double *__restrict__ dzf, int ny,
                                                 double *__restrict__ wsum_part)
{
    if (done && *done) return;
    extern __shared__ __align__(16) unsigned char smem[];
    const long line0 = (long)blockIdx.x * kDenseLines;
    const int k0 = (int)(line0 / ny), j0 = (int)(line0 - (long)k0 * ny);
    double acc = 0;
    auto src = [&](int e, int l) -> float {
        const long line = line0 + l;
        if (line >= nlines) return 0.f;
        const Tin x = in[line * n + e];
        if (wsum_part) acc += dzf[line_level(line, line0, k0, j0, ny)] * (double)x;
        return (float)x;
    };
    const double mp = EPI == 1 ? info[I_MEANP] : 0.0;
    auto put = [&](int q, int l, float v) {
        const long line = line0 + l;
        if (line < nlines) {
            const size_t idx = (size_t)line * n + q;
            if (EPI == 1) out[idx] = (Tout)((double)out[idx] + (double)v - mp);
            else out[idx] = (Tout)v;
        }
    };
    dense_transform(n, magn, src, put, Wh, Wl, reinterpret_cast<unsigned short *>(smem));
    if (wsum_part) {
        double z1 = 0, z2 = 0;
        block_sum3(acc, z1, z2);
        if (threadIdx.x == 0) {
            wsum_part[kNP * blockIdx.x] = acc;
        }
    }
}

__global__ __launch_bounds__(256) void k_dense_resid(const double *__restrict__ f, const double *__restrict__ p,
                                                     float *out, long nlines, int n, unsigned magn,
                                                     const unsigned short *__restrict__ Wh,
                                                     const unsigned short *__restrict__ Wl, LapArgs la,
                                                     const double *__restrict__ dzf,
                                                     const double *__restrict__ info,
                                                     double *__restrict__ partials, const int *__restrict__ done)
{
    if (*done) return;
    extern __shared__ __align__(16) unsigned char smem[];
    const int ny = la.ny;
    const long line0 = (long)blockIdx.x * kDenseLines;
    const int k0 = (int)(line0 / ny), j0 = (int)(line0 - (long)k0 * ny);
    const double mf = info[I_REMOVED];
    double srr = 0, sff = 0, spw = 0, rmax = 0, fmx = 0;
    auto src = [&](int e, int l) -> float {
        const long line = line0 + l;
        if (line >= nlines) return 0.f;
        const int k = line_level(line, line0, k0, j0, ny);
        const int j = (int)(line - (long)k * ny);
        const size_t gi = (size_t)line * n + e;
        const double fv = f[gi] - mf;
        const double r = fv - lap_point(p, e, j, k, la);
        srr += r * r;
        sff += fv * fv;
        rmax = fmax(rmax, fabs(r));
        fmx = fmax(fmx, fabs(fv));
        spw += dzf[k] * p[gi];
        return (float)r;
    };
    auto put = [&](int q, int l, float v) {
        const long line = line0 + l;
        if (line < nlines) out[(size_t)line * n + q] = v;
    };
    dense_transform(n, magn, src, put, Wh, Wl, reinterpret_cast<unsigned short *>(smem));
    put_partial(partials, blockIdx.x, srr, sff, spw, rmax, fmx);
}

static dim3 dense_grid(const Problem &pb)
{
    const long nlines = (long)pb.ny * pb.nz;
    return dim3((unsigned)((nlines + kDenseLines - 1) / kDenseLines));
}

// ---------------------------------------------------------------------------
// launchers
static size_t tile_lds(int axis, const XGeom &g, size_t elem) { return (size_t)tile_slots(axis, g) * 2 * elem; }

int launch_x_f64(const Problem &pb, bool fwd, const double *in, double *out, hipStream_t s)
{
    const XGeom &g = pb.ax.gx64[fwd ? 1 : 0];
    const long nlines = (long)pb.ny * pb.nz;
    const dim3 grid((unsigned)((nlines + g.L - 1) / g.L));
    const size_t sh = tile_lds(AX_X, g, sizeof(double));
    CANS_KIND_SWITCH(pb.ax.kind,
        if (fwd) hipLaunchKernelGGL((k_xform_x<KD, true, double, double, double, 0>), grid, dim3(kThreads), sh, s,
                                    in, out, nlines, g, pb.ax.d_tw64, nullptr, nullptr, nullptr, pb.ny, nullptr);
        else hipLaunchKernelGGL((k_xform_x<KD, false, double, double, double, 0>), grid, dim3(kThreads), sh, s,
                                in, out, nlines, g, pb.ax.d_tw64, nullptr, nullptr, nullptr, pb.ny, nullptr));
    return check_launch();
}

int launch_y_f64(const Problem &pb, bool fwd, const double *in, double *out, hipStream_t s)
{
    const XGeom &g = pb.ay.gy64[fwd ? 1 : 0];
    const int ntx = (pb.nx + g.L - 1) / g.L;
    const dim3 grid((unsigned)(ntx * pb.nz));
    const size_t sh = tile_lds(AX_Y, g, sizeof(double));
    CANS_KIND_SWITCH(pb.ay.kind,
        if (fwd) hipLaunchKernelGGL((k_xform_y<KD, true, double, double>), grid, dim3(kThreads), sh, s,
                                    in, out, pb.nx, pb.ny, ntx, g, pb.ay.d_tw64, nullptr);
        else hipLaunchKernelGGL((k_xform_y<KD, false, double, double>), grid, dim3(kThreads), sh, s,
                                in, out, pb.nx, pb.ny, ntx, g, pb.ay.d_tw64, nullptr));
    return check_launch();
}

// blocks of the first forward x transform, which also leaves the partial
// weighted sums of the rhs (one triple per block)
static int xfwd_blocks(const Problem &pb)
{
    const long nlines = (long)pb.ny * pb.nz;
    const int L = pb.ax.dense ? kDenseLines : pb.ax.gx32[1].L;
    return (int)((nlines + L - 1) / L);
}

int launch_x_fwd_32(const Problem &pb, const double *in, float *out, const int *done, hipStream_t s)
{
    if (pb.ax.dense) {
        hipLaunchKernelGGL((k_dense_x<true, double, float, 0>), dense_grid(pb), dim3(256), dense_lds(pb.nx), s, in, out,
                           (long)pb.ny * pb.nz, pb.nx, mag_of(pb.nx), pb.ax.d_wf_hi, pb.ax.d_wf_lo, nullptr, done,
                           pb.d_dzf, pb.ny, pb.partials);
        return check_launch();
    }
    const XGeom &g = pb.ax.gx32[1];
    const long nlines = (long)pb.ny * pb.nz;
    const dim3 grid((unsigned)xfwd_blocks(pb));
    const size_t sh = tile_lds(AX_X, g, sizeof(float));
    CANS_KIND_SWITCH(pb.ax.kind,
        hipLaunchKernelGGL((k_xform_x<KD, true, float, double, float, 0>), grid, dim3(kThreads), sh, s,
                           in, out, nlines, g, pb.ax.d_tw32, nullptr, done, pb.d_dzf, pb.ny, pb.partials));
    return check_launch();
}

int launch_y_32(const Problem &pb, bool fwd, float *data, const int *done, hipStream_t s)
{
    const XGeom &g = pb.ay.gy32[fwd ? 1 : 0];
    const int ntx = (pb.nx + g.L - 1) / g.L;
    const dim3 grid((unsigned)(ntx * pb.nz));
    const size_t sh = tile_lds(AX_Y, g, sizeof(float));
    CANS_KIND_SWITCH(pb.ay.kind,
        if (fwd) hipLaunchKernelGGL((k_xform_y<KD, true, float, float>), grid, dim3(kThreads), sh, s,
                                    data, data, pb.nx, pb.ny, ntx, g, pb.ay.d_tw32, done);
        else hipLaunchKernelGGL((k_xform_y<KD, false, float, float>), grid, dim3(kThreads), sh, s,
                                data, data, pb.nx, pb.ny, ntx, g, pb.ay.d_tw32, done));
    return check_launch();
}

int launch_x_inv_32(const Problem &pb, const float *in, double *p, bool update, const int *done,
                    hipStream_t s)
{
    if (pb.ax.dense) {
        if (update)
            hipLaunchKernelGGL((k_dense_x<false, float, double, 1>), dense_grid(pb), dim3(256), dense_lds(pb.nx), s,
                               in, p, (long)pb.ny * pb.nz, pb.nx, mag_of(pb.nx), pb.ax.d_wi_hi, pb.ax.d_wi_lo,
                               pb.d_info, done, nullptr, pb.ny, nullptr);
        else
            hipLaunchKernelGGL((k_dense_x<false, float, double, 0>), dense_grid(pb), dim3(256), dense_lds(pb.nx), s,
                               in, p, (long)pb.ny * pb.nz, pb.nx, mag_of(pb.nx), pb.ax.d_wi_hi, pb.ax.d_wi_lo,
                               pb.d_info, done, nullptr, pb.ny, nullptr);
        return check_launch();
    }
    const XGeom &g = pb.ax.gx32[0];
    const long nlines = (long)pb.ny * pb.nz;
    const dim3 grid((unsigned)((nlines + g.L - 1) / g.L));
    const size_t sh = tile_lds(AX_X, g, sizeof(float));
    CANS_KIND_SWITCH(pb.ax.kind,
        if (update) hipLaunchKernelGGL((k_xform_x<KD, false, float, float, double, 1>), grid, dim3(kThreads), sh, s,
                                       in, p, nlines, g, pb.ax.d_tw32, pb.d_info, done, nullptr, pb.ny, nullptr);
        else hipLaunchKernelGGL((k_xform_x<KD, false, float, float, double, 0>), grid, dim3(kThreads), sh, s,
                                in, p, nlines, g, pb.ax.d_tw32, pb.d_info, done, nullptr, pb.ny, nullptr));
    return check_launch();
}

static ZArgs zargs(const Problem &pb, double *removed)
{
    ZArgs a;
    a.nx = pb.nx; a.ny = pb.ny; a.nz = pb.nz;
    a.za = pb.d_za; a.zb = pb.d_zb; a.zc = pb.d_zc;
    a.lamx = pb.ax.d_lam; a.lamy = pb.ay.d_lam;
    a.dzf = pb.d_dzf; a.wsum = pb.wsum; a.scale = pb.scale;
    a.cyclic = pb.cyclic; a.singular = pb.singular;
    a.wc = pb.wc; a.wd = pb.wd; a.wz = pb.wz;
    a.removed = removed;
    return a;
}

int launch_zsolve_f64(const Problem &pb, double *data, double *removed, hipStream_t s)
{
    return launch_zsolve<double>(pb, data, removed, nullptr, s);
}

int launch_zsolve_32(const Problem &pb, float *data, double *removed, const int *done, hipStream_t s)
{
    return launch_zsolve<float>(pb, data, removed, done, s);
}

static LapArgs lapargs(const Problem &pb)
{
    LapArgs la;
    la.nx = pb.nx; la.ny = pb.ny; la.nz = pb.nz;
    for (int i = 0; i < 6; ++i) la.bc[i] = pb.bc[i];
    la.idx2 = 1.0 / (pb.ax.h * pb.ax.h);
    la.idy2 = 1.0 / (pb.ay.h * pb.ay.h);
    la.zaf = pb.d_zaf; la.zcf = pb.d_zcf;
    la.shift = pb.shift;
    return la;
}

int resid_blocks(const Problem &pb)
{
    const long nlines = (long)pb.ny * pb.nz;
    const int L = pb.ax.dense ? kDenseLines : pb.ax.gx32[1].L;
    return (int)((nlines + L - 1) / L);
}

int launch_resid_xfwd(const Problem &pb, const double *f, const double *p, float *out, const int *done,
                      hipStream_t s)
{
    if (pb.ax.dense) {
        hipLaunchKernelGGL(k_dense_resid, dense_grid(pb), dim3(256), dense_lds(pb.nx), s, f, p, out,
                           (long)pb.ny * pb.nz, pb.nx, mag_of(pb.nx), pb.ax.d_wf_hi, pb.ax.d_wf_lo, lapargs(pb),
                           pb.d_dzf, pb.d_info, pb.partials, done);
        return check_launch();
    }
    const XGeom &g = pb.ax.gx32[1];
    const long nlines = (long)pb.ny * pb.nz;
    const dim3 grid((unsigned)resid_blocks(pb));
    const size_t sh = tile_lds(AX_X, g, sizeof(float));
    CANS_KIND_SWITCH(pb.ax.kind,
        hipLaunchKernelGGL(k_resid_xfwd<KD>, grid, dim3(kThreads), sh, s, f, p, out, nlines, g,
                           pb.ax.d_tw32, lapargs(pb), pb.d_dzf, pb.d_info, pb.partials, done));
    return check_launch();
}

int launch_resid_norm(const Problem &pb, const double *f, const double *p, const int *done, hipStream_t s)
{
    const long nlines = (long)pb.ny * pb.nz;
    hipLaunchKernelGGL(k_resid_norm, dim3((unsigned)resid_blocks(pb)), dim3(kThreads), 0, s, f, p, nlines,
                       pb.ax.dense ? kDenseLines : pb.ax.gx32[1].L, lapargs(pb), pb.d_dzf, pb.d_info, pb.partials, done);
    return check_launch();
}

// Up to this many block partials the last-level kernel reads them directly
// (one launch per check instead of two; small problems are launch-bound).
constexpr int kDirectReduce = 4096;

int launch_finalize(const Problem &pb, int check, int max_iter, double tol, hipStream_t s)
{
    const double inv_wvol = 1.0 / (pb.wsum * pb.nx * pb.ny);
    const int nblk = resid_blocks(pb);
    if (nblk <= kDirectReduce) {
        hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kThreads), 0, s, pb.partials, nblk, check, max_iter, tol,
                           inv_wvol, pb.singular, pb.d_info, pb.d_flag);
        return check_launch();
    }
    hipLaunchKernelGGL(k_reduce1, dim3(kReduceBlocks), dim3(kThreads), 0, s, pb.partials, nblk, pb.sums,
                       pb.d_flag);
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kThreads), 0, s, pb.sums, kReduceBlocks, check, max_iter, tol,
                       inv_wvol, pb.singular, pb.d_info, pb.d_flag);
    return check_launch();
}

int launch_mean_rhs(const Problem &pb, hipStream_t s)
{
    const double inv_wvol = 1.0 / (pb.wsum * pb.nx * pb.ny);
    const int nblk = xfwd_blocks(pb);
    if (nblk <= kDirectReduce) {
        hipLaunchKernelGGL(k_mean_rhs, dim3(1), dim3(kThreads), 0, s, pb.partials, nblk, inv_wvol, pb.singular,
                           pb.d_info);
        return check_launch();
    }
    hipLaunchKernelGGL(k_reduce1, dim3(kReduceBlocks), dim3(kThreads), 0, s, pb.partials, nblk, pb.sums, nullptr);
    hipLaunchKernelGGL(k_mean_rhs, dim3(1), dim3(kThreads), 0, s, pb.sums, kReduceBlocks, inv_wvol, pb.singular,
                       pb.d_info);
    return check_launch();
}

int launch_reset(const Problem &pb, hipStream_t s)
{
    hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, s, pb.d_info, pb.d_flag);
    return check_launch();
}

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

// k_resid.hip -- FP64 residual of eq. (poi) for iterative refinement (fused with the forward
// x transform, or norms only), the fixed-order reductions that decide convergence, and their launchers.
#include "kcommon.h"

namespace cans {

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


int resid_blocks(const Problem &pb)
{
    const long nlines = (long)pb.ny * pb.nz;
    const int L = pb.ax.dense ? kDenseLines : pb.ax.gx32[1].L;
    return (int)((nlines + L - 1) / L);
}

int launch_resid_xfwd(const Problem &pb, const Work &w, const double *f, const double *p, float *out,
                      const int *done, hipStream_t s)
{
    if (pb.ax.dense) {
        hipLaunchKernelGGL(k_dense_resid, dense_grid(pb), dim3(256), dense_lds(pb.nx), s, f, p, out,
                           (long)pb.ny * pb.nz, pb.nx, mag_of(pb.nx), pb.ax.d_wf_hi, pb.ax.d_wf_lo, lapargs(pb),
                           pb.d_dzf, w.info, w.partials, done);
        return check_launch();
    }
    const XGeom &g = pb.ax.gx32[1];
    const long nlines = (long)pb.ny * pb.nz;
    const dim3 grid((unsigned)resid_blocks(pb));
    const size_t sh = tile_lds(AX_X, g, sizeof(float));
    CANS_KIND_SWITCH(pb.ax.kind,
        hipLaunchKernelGGL(k_resid_xfwd<KD>, grid, dim3(kThreads), sh, s, f, p, out, nlines, g,
                           pb.ax.d_tw32, lapargs(pb), pb.d_dzf, w.info, w.partials, done));
    return check_launch();
}

int launch_resid_norm(const Problem &pb, const Work &w, const double *f, const double *p, const int *done,
                      hipStream_t s)
{
    const long nlines = (long)pb.ny * pb.nz;
    hipLaunchKernelGGL(k_resid_norm, dim3((unsigned)resid_blocks(pb)), dim3(kThreads), 0, s, f, p, nlines,
                       pb.ax.dense ? kDenseLines : pb.ax.gx32[1].L, lapargs(pb), pb.d_dzf, w.info, w.partials, done);
    return check_launch();
}

// Up to this many block partials the last-level kernel reads them directly
// (one launch per check instead of two; small problems are launch-bound).
constexpr int kDirectReduce = 4096;

int launch_finalize(const Problem &pb, const Work &w, int check, int max_iter, double tol, hipStream_t s)
{
    const double inv_wvol = 1.0 / (pb.wsum * pb.nx * pb.ny);
    const int nblk = resid_blocks(pb);
    if (nblk <= kDirectReduce) {
        hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kThreads), 0, s, w.partials, nblk, check, max_iter, tol,
                           inv_wvol, pb.singular, w.info, w.flag);
        return check_launch();
    }
    hipLaunchKernelGGL(k_reduce1, dim3(kReduceBlocks), dim3(kThreads), 0, s, w.partials, nblk, w.sums,
                       w.flag);
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kThreads), 0, s, w.sums, kReduceBlocks, check, max_iter, tol,
                       inv_wvol, pb.singular, w.info, w.flag);
    return check_launch();
}

int launch_mean_rhs(const Problem &pb, const Work &w, hipStream_t s)
{
    const double inv_wvol = 1.0 / (pb.wsum * pb.nx * pb.ny);
    const int nblk = xfwd_blocks(pb);
    if (nblk <= kDirectReduce) {
        hipLaunchKernelGGL(k_mean_rhs, dim3(1), dim3(kThreads), 0, s, w.partials, nblk, inv_wvol, pb.singular,
                           w.info);
        return check_launch();
    }
    hipLaunchKernelGGL(k_reduce1, dim3(kReduceBlocks), dim3(kThreads), 0, s, w.partials, nblk, w.sums, nullptr);
    hipLaunchKernelGGL(k_mean_rhs, dim3(1), dim3(kThreads), 0, s, w.sums, kReduceBlocks, inv_wvol, pb.singular,
                       w.info);
    return check_launch();
}

__global__ void k_clear_work(double *__restrict__ info, int *__restrict__ flag, unsigned *__restrict__ zctr)
{
    const int t = threadIdx.x;
    if (t < I_SIZE) info[t] = 0.0;
    if (t == 0) flag[0] = 0;
    if (zctr && t < 2) zctr[t] = 0u;
}

__global__ void k_copy_info(const double *__restrict__ src, double *__restrict__ dst)
{
    const int t = threadIdx.x;
    if (t < I_SIZE) dst[t] = src[t];
}

int launch_clear_work(const Work &w, hipStream_t s)
{
    hipLaunchKernelGGL(k_clear_work, dim3(1), dim3(64), 0, s, w.info, w.flag, w.zctr);
    return check_launch();
}

int launch_copy_info(const double *src, double *dst, hipStream_t s)
{
    hipLaunchKernelGGL(k_copy_info, dim3(1), dim3(64), 0, s, src, dst);
    return check_launch();
}

int launch_reset(const Problem &pb, const Work &w, hipStream_t s)
{
    hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, s, w.info, w.flag);
    return check_launch();
}
}  // namespace cans

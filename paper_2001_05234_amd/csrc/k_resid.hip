// k_resid.hip -- FP64 residual of eq. (poi) for iterative refinement (fused with the forward
// x transform, or norms only), the fixed-order reductions that decide convergence, and their launchers.
#include "kcommon.h"

namespace cans {

// ---------------------------------------------------------------------------
// Residual kernels.  A block takes L consecutive rows (x lines) of one plane.
// Block b belongs to XCD b % 8 (blocks are dispatched round-robin over the
// eight XCDs); XCD x owns the rows [x H, (x+1) H) of every plane and walks
// them plane by plane, so the rows above and below a block's rows (y
// neighbours) and the same rows one plane up and down (z neighbours) are read
// by the same XCD close in time and come from its L2: each p value reaches
// HBM about once.  H is ceil(ny/8) rounded up to a multiple of L.
// Short rows (nx <= kFlatMaxN) take the flat form instead: block b takes the
// L consecutive rows (x lines j + ny k, across planes) from b L on, and forms
// their residual in groups of up to G rows of one plane spread over the
// block's threads (a slice of a small grid would leave most XCDs idle, and a
// short row most threads).  RSlice.H = 0 marks it, with bpp = G.
struct RSlice {
    int L, H, bpp;   // rows per block, slice height, blocks per plane and slice (flat: 0, G)
};

constexpr int kFlatMaxN = 512;
constexpr int kResidU = 4;                       // points of a row per thread and chunk
constexpr int kResidChunk = kResidU * kThreads;  // 1024
constexpr int kRowsD = 2 * (kResidChunk + 4);    // doubles of the `rows` LDS buffer (either form)

// rows of a flat group: as many as fill a chunk, with their two neighbour
// rows and ghosts inside `rows`
static __host__ __device__ inline int flat_group(int n)
{
    const int g1 = kResidChunk / n, g2 = kRowsD / (n + 2) - 2;
    const int g = g1 < g2 ? g1 : g2;
    return g > 1 ? g : 1;
}

static inline RSlice rslice(const Problem &pb, int L)
{
    if (pb.nx <= kFlatMaxN) return RSlice{L, 0, flat_group(pb.nx)};
    const int h8 = (pb.ny + 7) / 8;
    const int H = (h8 + L - 1) / L * L;
    return RSlice{L, H, H / L};
}

static inline int rslice_blocks(const Problem &pb, const RSlice &rs)
{
    if (rs.H == 0) return (int)(((long)pb.ny * pb.nz + rs.L - 1) / rs.L);
    return 8 * pb.nz * rs.bpp;
}

// rows of the norm-only kernel (x lines per block): two of a long row; of
// short rows (the flat form) four groups when the problem still has 1024
// blocks or more (a block's closing reduction then serves four groups), else
// one
static inline int norm_rows(const Problem &pb)
{
    if (pb.nx > kFlatMaxN) return 2;
    const int G = flat_group(pb.nx);
    const long groups = ((long)pb.ny * pb.nz + G - 1) / G;
    return groups >= 4096 ? 4 * G : G;
}

// rows of exactly one chunk take the kernels' exact form
static inline bool exact_rows(const Problem &pb) { return pb.nx == kResidChunk; }

// The residual r = (f - mf) - L_h p (eq. (poi), plus the plan's shift) of the
// rows j0 .. j0 + nr - 1 (nr <= 2) of plane k, block-wide, in chunks of
// kResidChunk points of a row.  Each thread first loads all it needs of the
// chunk into registers: its kResidU points of the two rows and of the rows
// just below and above them (by the y rule of `beyond` at a domain
// boundary: periodic wraps, Neumann mirrors, Dirichlet mirrors with the sign
// flipped; a face-located field is zero beyond a Dirichlet face and mirrored
// about a Neumann face), so every global load is in flight at once.  The rows themselves
// go to LDS (`rows`, 2 (kResidChunk + 2) of its kRowsD doubles) for the x neighbours; the
// planes above and below and f are loaded after the barrier, again all at
// once.  The arithmetic per point is lap_point's.  put(l, e, r) receives every
// residual; acc accumulates the block's partial sums.
struct RAcc {
    double srr = 0, sff = 0, spw = 0, rmax = 0, fmx = 0;
};

// EXACT: rows of exactly kResidChunk points (one chunk, no bounds to check).
template <bool EXACT, typename Put>
__device__ void resid_pair(const double *__restrict__ f, const double *__restrict__ p, int k, int j0, int nr,
                           const LapArgs &la, double mf, double wk, double *rows, Put put, RAcc &acc)
{
    const int n = EXACT ? kResidChunk : la.nx, ny = la.ny, nz = la.nz;
    const size_t sy = (size_t)n, sz = (size_t)n * ny;
    const double *pk = p + sz * k;
    const int t = (int)threadIdx.x, rs = kResidChunk + 2;
    // the staged rows: 0 = j0 - 1, 1 = j0, 2 = j0 + 1 (if nr == 2), nr + 1 = above
    const double *rp[4];
    double sg[4];
    for (int l = 0; l < 4; ++l) {
        int j = j0 + l - 1;
        if (l == nr + 1) j = j0 + nr;
        if (l > nr + 1) j = j0 + nr - 1;  // not used
        sg[l] = 1.0;
        if (j < 0) beyond(la.bc[2], true, ny, j, sg[l]);
        else if (j >= ny) beyond(la.bc[3], false, ny, j, sg[l]);
        rp[l] = pk + sy * j;
    }
    // the planes below and above; at a wall the plane itself with the sign of
    // its ghost rule (Neumann +, Dirichlet and the face-located z field -),
    // so every point takes one multiply instead of a select
    const double *zm_pl = k > 0 ? pk - sz : (la.bc[4] == 0 ? p + sz * (nz - 1) : pk);
    const double *zp_pl = k < nz - 1 ? pk + sz : (la.bc[5] == 0 ? p : pk);
    const double gzm = (k > 0 || la.bc[4] <= 1) ? 1.0 : -1.0, gzp = (k < nz - 1 || la.bc[5] <= 1) ? 1.0 : -1.0;
    const double zaf = la.zaf[k], zcf = la.zcf[k];
    const double *fk = f + sz * k;
    for (int e0 = 0; e0 < n; e0 += kResidChunk) {
        // unconditional loads (indices clamped into the row) so that they
        // are all issued before the first wait
        double c[4][kResidU];
#pragma unroll
        for (int l = 0; l < 4; ++l)
#pragma unroll
            for (int u = 0; u < kResidU; ++u) {
                const int e = e0 + t + u * kThreads;
                c[l][u] = sg[l] * rp[l][EXACT || e < n ? e : n - 1];
            }
        __syncthreads();  // the previous chunk's reads of `rows` are done
        // the rows' chunk in LDS, with the x neighbours just outside it
#pragma unroll
        for (int l = 0; l < 2; ++l)
#pragma unroll
            for (int u = 0; u < kResidU; ++u) {
                const int e = e0 + t + u * kThreads;
                if (EXACT || e < n) rows[l * rs + 1 + t + u * kThreads] = c[l + 1][u];
            }
        if (t < 2 * 2) {
            // x neighbours just outside the chunk: the next chunk's first
            // point, or the ghost after the row's last point
            const int l = t >> 1;
            if (l < nr) {
                const double *row = rp[l + 1];
                if ((t & 1) == 0)
                    rows[l * rs] = e0 > 0 ? row[e0 - 1] : across(la.bc[0], true, row, 0, 0, n, 1);
                else if (e0 + kResidChunk < n)
                    rows[l * rs + kResidChunk + 1] = row[e0 + kResidChunk];
                else
                    rows[l * rs + 1 + (n - e0)] = across(la.bc[1], false, row, n - 1, n - 1, n, 1);
            }
        }
        __syncthreads();
#pragma unroll
        for (int l = 0; l < 2; ++l) {
            if (l >= nr) break;
            // the planes above and below and f of the row's points, all in flight at once
            double zmv[kResidU], zpv[kResidU], fvv[kResidU];
            const size_t ro = sy * (j0 + l);
#pragma unroll
            for (int u = 0; u < kResidU; ++u) {
                const int e = e0 + t + u * kThreads;
                const size_t o = ro + (EXACT || e < n ? e : 0);
                zmv[u] = zm_pl[o];
                zpv[u] = zp_pl[o];
                fvv[u] = fk[o];
            }
#pragma unroll
            for (int u = 0; u < kResidU; ++u) {
                const int e = e0 + t + u * kThreads;
                const int q = 1 + t + u * kThreads;
                if (EXACT || e < n) {
                    const double cc = c[l + 1][u];
                    const double xm = rows[l * rs + q - 1], xp = rows[l * rs + q + 1];
                    const double ym = c[l][u], yp = c[l + 2][u];
                    const double zm = gzm * zmv[u], zp = gzp * zpv[u];
                    const double fv = fvv[u] - mf;
                    const double lap = (xm - 2.0 * cc + xp) * la.idx2 + (ym - 2.0 * cc + yp) * la.idy2 +
                                       zcf * (zp - cc) - zaf * (cc - zm) + la.shift * cc;
                    const double r = fv - lap;
                    put(l, e, r);
                    acc.srr += r * r;
                    acc.sff += fv * fv;
                    acc.rmax = fmax(acc.rmax, fabs(r));
                    acc.fmx = fmax(acc.fmx, fabs(fv));
                    acc.spw += wk * cc;
                }
            }
        }
    }
    __syncthreads();  // `rows` free for the caller
}

// block -> (plane, first row, rows in the plane); lv = 0 for a block beyond the grid
static __device__ inline void rslice_of(unsigned b, int H, int bpp, int L, int ny, int nz, int &k, int &j0, int &lv)
{
    const int x = (int)(b % 8), i = (int)(b / 8);
    k = i / bpp;
    j0 = x * H + (i % bpp) * L;
    lv = (k < nz && j0 < ny) ? min(L, ny - j0) : 0;
}

// The flat form of the residual: rows j0 .. j0 + nr - 1 of plane k with
// nr nx <= kResidChunk, one point per thread and slot.  The nr rows and the
// rows next to them (by the y rule of `beyond`) go to `rows` first (stride
// nx + 2, an x ghost at each end), every load in flight at once; then the x
// ghosts; then each thread loads the planes above and below and f of its
// points, all at once, and forms lap_point's expression from LDS.
template <typename Put>
__device__ void resid_rows_flat(const double *__restrict__ f, const double *__restrict__ p, int k, int j0, int nr,
                                const LapArgs &la, double mf, double wk, double *rows, Put put, RAcc &acc)
{
    const int n = la.nx, ny = la.ny, nz = la.nz;
    const size_t sy = (size_t)n, sz = (size_t)n * ny;
    const double *pk = p + sz * k;
    const int t = (int)threadIdx.x, rs = n + 2;
    const unsigned mag = mag_of((unsigned)n);
    // the rows next to the group: ordinary rows, or by the y rule beyond a face
    int jlo = j0 - 1, jhi = j0 + nr;
    double slo = 1.0, shi = 1.0;
    if (jlo < 0) beyond(la.bc[2], true, ny, jlo, slo);
    if (jhi >= ny) beyond(la.bc[3], false, ny, jhi, shi);
    constexpr int SU = 2 * kResidU;  // (nr + 2) nx <= kResidChunk + 2 kFlatMaxN values, SU a thread
    const int tot = (nr + 2) * n;
    double v[SU];
#pragma unroll
    for (int u = 0; u < SU; ++u) {
        const int idx = min(t + u * kThreads, tot - 1);  // clamped: every load issued unconditionally
        const int r = (int)udiv((unsigned)idx, (unsigned)n, mag), e = idx - r * n;
        const int j = r == 0 ? jlo : (r == nr + 1 ? jhi : j0 + r - 1);
        const double sg = r == 0 ? slo : (r == nr + 1 ? shi : 1.0);
        v[u] = sg * pk[sy * j + e];
    }
#pragma unroll
    for (int u = 0; u < SU; ++u) {
        const int idx = t + u * kThreads;
        if (idx < tot) {
            const int r = (int)udiv((unsigned)idx, (unsigned)n, mag), e = idx - r * n;
            rows[r * rs + 1 + e] = v[u];
        }
    }
    __syncthreads();
    if (t < 2 * nr) {  // x ghosts of the group's own rows
        double *row = rows + (1 + (t >> 1)) * rs + 1;
        if ((t & 1) == 0) row[-1] = across(la.bc[0], true, row, 0, 0, n, 1);
        else row[n] = across(la.bc[1], false, row, n - 1, n - 1, n, 1);
    }
    __syncthreads();
    // the planes below and above; at a wall the plane itself with the sign of
    // its ghost rule (Neumann +, Dirichlet and the face-located z field -),
    // so every point takes one multiply instead of a select
    const double *zm_pl = k > 0 ? pk - sz : (la.bc[4] == 0 ? p + sz * (nz - 1) : pk);
    const double *zp_pl = k < nz - 1 ? pk + sz : (la.bc[5] == 0 ? p : pk);
    const double gzm = (k > 0 || la.bc[4] <= 1) ? 1.0 : -1.0, gzp = (k < nz - 1 || la.bc[5] <= 1) ? 1.0 : -1.0;
    const double zaf = la.zaf[k], zcf = la.zcf[k];
    const double *fk = f + sz * k;
    const int np = nr * n;
    double zmv[kResidU], zpv[kResidU], fvv[kResidU];
    int rr[kResidU], ee[kResidU];
#pragma unroll
    for (int u = 0; u < kResidU; ++u) {
        const int idx = min(t + u * kThreads, np - 1);
        const int r = (int)udiv((unsigned)idx, (unsigned)n, mag), e = idx - r * n;
        rr[u] = r;
        ee[u] = e;
        const size_t o = sy * (j0 + r) + e;
        zmv[u] = zm_pl[o];
        zpv[u] = zp_pl[o];
        fvv[u] = fk[o];
    }
#pragma unroll
    for (int u = 0; u < kResidU; ++u) {
        if (t + u * kThreads < np) {
            const double *q = rows + (rr[u] + 1) * rs + 1 + ee[u];
            const double cc = q[0];
            const double xm = q[-1], xp = q[1], ym = q[-rs], yp = q[rs];
            const double zm = gzm * zmv[u], zp = gzp * zpv[u];
            const double fv = fvv[u] - mf;
            const double lap = (xm - 2.0 * cc + xp) * la.idx2 + (ym - 2.0 * cc + yp) * la.idy2 +
                               zcf * (zp - cc) - zaf * (cc - zm) + la.shift * cc;
            const double r = fv - lap;
            put(rr[u], ee[u], r);
            acc.srr += r * r;
            acc.sff += fv * fv;
            acc.rmax = fmax(acc.rmax, fabs(r));
            acc.fmx = fmax(acc.fmx, fabs(fv));
            acc.spw += wk * cc;
        }
    }
    __syncthreads();  // `rows` free for the next group
}

// The residual rows of block blk in either mapping (H > 0: XCD slices, rows
// of one plane in pairs; H = 0: flat, bpp = G rows a group).  put(l, e, r)
// receives line l of the block; line0 and lv give its first line and count.
// EX: the slice mapping over rows of exactly kResidChunk points only (its own
// kernels, so that the general paths do not raise their register count).
template <bool EX, typename Put>
__device__ __forceinline__ void resid_block(const double *__restrict__ f, const double *__restrict__ p, int H,
                                            int bpp, int L, const LapArgs &la, double mf,
                                            const double *__restrict__ dzf, double *rows, unsigned blk, Put put,
                                            RAcc &acc, long &line0, int &lv)
{
    const int ny = la.ny;
    if (EX || H > 0) {
        int k, j0;
        rslice_of(blk, H, bpp, L, ny, la.nz, k, j0, lv);
        line0 = (long)k * ny + j0;
        for (int l0 = 0; l0 < lv; l0 += 2)
            resid_pair<EX>(f, p, k, j0 + l0, min(2, lv - l0), la, mf, dzf[k], rows,
                           [&](int l, int e, double r) { put(l0 + l, e, r); }, acc);
        return;
    }
    const long nlines = (long)ny * la.nz;
    line0 = (long)blk * L;
    lv = line0 < nlines ? (int)min((long)L, nlines - line0) : 0;
    for (int l0 = 0; l0 < lv;) {
        const long line = line0 + l0;
        const int k = (int)(line / ny), j = (int)(line - (long)k * ny);
        const int nr = min(min(bpp, lv - l0), ny - j);
        resid_rows_flat(f, p, k, j, nr, la, mf, dzf[k], rows, [&](int l, int e, double r) { put(l0 + l, e, r); },
                        acc);
        l0 += nr;
    }
}

// The residual fused with the forward x transform of its rows (FP32 out);
// block partials: sums of |r|^2, |f - mean|^2, dzf p; maxima of |r|, |f - mean|.
// The bodies take the block index, so that one launch can serve one problem
// (blk = blockIdx.x) or a group of problems (the *_grp kernels).
template <int KIND, bool EX>
__device__ __forceinline__ void resid_xfwd_body(const double *__restrict__ f, const double *__restrict__ p,
                                                float *out, int H, int bpp, const XGeom &g, int rows_off,
                                                const cx<float> *__restrict__ tw, const LapArgs &la,
                                                const double *__restrict__ dzf, const double *__restrict__ info,
                                                double *__restrict__ partials, const int *__restrict__ done,
                                                unsigned blk)
{
    if (*done) return;
    extern __shared__ __align__(16) unsigned char smem[];
    const Tile<AX_X, float> tile{reinterpret_cast<cx<float> *>(smem), g.L, g.RS, g.psh};
    double *rows = reinterpret_cast<double *>(smem + rows_off);  // after the transform tile
    const int n = g.nl, L = g.L;
    RAcc acc;
    long line0;
    int lv;
    resid_block<EX>(f, p, H, bpp, L, la, info[I_REMOVED], dzf, rows, blk,
                    [&](int l, int e, double r) { tile_real(tile, e, l) = (float)r; }, acc, line0, lv);
    if (lv > 0) {
        for (int idx = threadIdx.x; idx < (L - lv) * n; idx += kThreads)
            tile_real(tile, idx % n, lv + idx / n) = 0.f;
        __syncthreads();
        auto src = [&](int e, int l) -> float { return tile_real(tile, e, l); };
        auto put = [&](int q, int l, float v) {
            if (l < lv) out[(size_t)(line0 + l) * n + q] = v;
        };
        tile_transform<KIND, true, AX_X, true, true>(threadIdx.x, kThreads, g, src, put, tile, tile, tw, BlockSync());
    }
    put_partial(partials, blk, acc.srr, acc.sff, acc.spw, acc.rmax, acc.fmx);
}

template <int KIND, bool EX>
__global__ __launch_bounds__(kThreads) void k_resid_xfwd(const double *__restrict__ f,
                                                         const double *__restrict__ p, float *out, int H, int bpp,
                                                         XGeom g, int rows_off, const cx<float> *__restrict__ tw,
                                                         LapArgs la,
                                                         const double *__restrict__ dzf,
                                                         const double *__restrict__ info,
                                                         double *__restrict__ partials,
                                                         const int *__restrict__ done)
{
    resid_xfwd_body<KIND, EX>(f, p, out, H, bpp, g, rows_off, tw, la, dzf, info, partials, done, blockIdx.x);
}

// Residual norms only (the check after a correction): the same block
// partials over norm_rows() rows a block.
template <bool EX>
__device__ __forceinline__ void resid_norm_body(const double *__restrict__ f, const double *__restrict__ p, int H,
                                                int bpp, int L, const LapArgs &la, const double *__restrict__ dzf,
                                                const double *__restrict__ info, double *__restrict__ partials,
                                                const int *__restrict__ done, unsigned blk)
{
    if (*done) return;
    extern __shared__ __align__(16) unsigned char smem[];
    double *rows = reinterpret_cast<double *>(smem);
    RAcc acc;
    long line0;
    int lv;
    resid_block<EX>(f, p, H, bpp, L, la, info[I_REMOVED], dzf, rows, blk, [](int, int, double) {}, acc, line0, lv);
    put_partial(partials, blk, acc.srr, acc.sff, acc.spw, acc.rmax, acc.fmx);
}

template <bool EX>
__global__ __launch_bounds__(kThreads) void k_resid_norm(const double *__restrict__ f,
                                                         const double *__restrict__ p, int H, int bpp, int L,
                                                         LapArgs la, const double *__restrict__ dzf,
                                                         const double *__restrict__ info,
                                                         double *__restrict__ partials,
                                                         const int *__restrict__ done)
{
    resid_norm_body<EX>(f, p, H, bpp, L, la, dzf, info, partials, done, blockIdx.x);
}


template <int KIND, bool EX>
__global__ __launch_bounds__(kThreads) void k_resid_xfwd_grp(const RJob *__restrict__ jobs,
                                                             const unsigned *__restrict__ start, int np)
{
    const int q = group_find(start, np, blockIdx.x);
    const RJob &j = jobs[q];
    const unsigned blk = blockIdx.x - start[q];
    if (blk >= j.nblk) return;
    resid_xfwd_body<KIND, EX>(j.f, j.p, j.out, j.H, j.bpp, j.g, j.rows_off, static_cast<const cx<float> *>(j.tw), j.la,
                          j.dzf, j.info, j.partials, j.done, blk);
}

template <bool EX>
__global__ __launch_bounds__(kThreads) void k_resid_norm_grp(const RJob *__restrict__ jobs,
                                                             const unsigned *__restrict__ start, int np)
{
    const int q = group_find(start, np, blockIdx.x);
    const RJob &j = jobs[q];
    const unsigned blk = blockIdx.x - start[q];
    if (blk >= j.nblk) return;
    resid_norm_body<EX>(j.f, j.p, j.H, j.bpp, j.L, j.la, j.dzf, j.info, j.partials, j.done, blk);
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
__device__ __forceinline__ void finalize_body(const double *__restrict__ partials, int nblk, int check, int max_iter,
                                              double tol, double inv_wvol, int singular, double *__restrict__ info,
                                              int *__restrict__ flag)
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

__global__ __launch_bounds__(kThreads) void k_finalize(const double *__restrict__ partials, int nblk,
                                                       int check, int max_iter, double tol,
                                                       double inv_wvol, int singular,
                                                       double *__restrict__ info, int *__restrict__ flag)
{
    finalize_body(partials, nblk, check, max_iter, tol, inv_wvol, singular, info, flag);
}

// Exact FP64 weighted mean of the rhs from the first pass's block sums:
// info[I_REMOVED] = sum dzf f / (nx ny sum dzf) when singular, else 0.
__device__ __forceinline__ void mean_rhs_body(const double *__restrict__ partials, int nblk, double inv_wvol,
                                              int singular, double *__restrict__ info)
{
    double a = 0, b = 0, c = 0;
    for (int i = threadIdx.x; i < nblk; i += kThreads) a += partials[(size_t)kNP * i];
    block_sum3(a, b, c);
    if (threadIdx.x == 0) info[I_REMOVED] = singular ? a * inv_wvol : 0.0;
}

__global__ __launch_bounds__(kThreads) void k_mean_rhs(const double *__restrict__ partials, int nblk,
                                                       double inv_wvol, int singular,
                                                       double *__restrict__ info)
{
    mean_rhs_body(partials, nblk, inv_wvol, singular, info);
}

// Start-of-solve state, written by a kernel so the sequence can be captured.
__global__ void k_reset(double *__restrict__ info, int *__restrict__ flag)
{
    const int t = threadIdx.x;
    if (t < I_SIZE) info[t] = (t >= I_HIST || t == I_LAST) ? -1.0 : 0.0;
    if (t == 0) flag[0] = 0;
}

// The per-problem reductions of a grouped batch, one block per problem:
// start-of-solve state, the rhs mean after the first x transform, and the
// check after a residual pass (which = 0: the fused pass's partials, 1: the
// norm pass's).
__global__ __launch_bounds__(kThreads) void k_reset_grp(const FJob *__restrict__ jobs)
{
    const FJob &j = jobs[blockIdx.x];
    const int t = threadIdx.x;
    if (t < I_SIZE) j.info[t] = (t >= I_HIST || t == I_LAST) ? -1.0 : 0.0;
    if (t == 0) j.flag[0] = 0;
}

__global__ __launch_bounds__(kThreads) void k_mean_rhs_grp(const FJob *__restrict__ jobs)
{
    const FJob &j = jobs[blockIdx.x];
    mean_rhs_body(j.partials, j.nb_mean, j.inv_wvol, j.singular, j.info);
}

__global__ __launch_bounds__(kThreads) void k_finalize_grp(const FJob *__restrict__ jobs, int which, int check,
                                                           int max_iter, double tol)
{
    const FJob &j = jobs[blockIdx.x];
    finalize_body(j.partials, which == 0 ? j.nb_xfwd : j.nb_norm, check, max_iter, tol, j.inv_wvol, j.singular,
                  j.info, j.flag);
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


int resid_blocks_xfwd(const Problem &pb)
{
    if (pb.ax.dense) return (int)dense_grid(pb).x;
    return rslice_blocks(pb, rslice(pb, pb.ax.gxr32.L));
}

int resid_blocks_norm(const Problem &pb) { return rslice_blocks(pb, rslice(pb, norm_rows(pb))); }

int launch_resid_xfwd(const Problem &pb, const Work &w, const double *f, const double *p, float *out,
                      const int *done, hipStream_t s)
{
    if (pb.ax.dense) {
        hipLaunchKernelGGL(k_dense_resid, dense_grid(pb), dim3(256), dense_lds(pb.nx), s, f, p, out,
                           (long)pb.ny * pb.nz, pb.nx, mag_of(pb.nx), pb.ax.d_wf_hi, pb.ax.d_wf_lo, lapargs(pb),
                           pb.d_dzf, w.info, w.partials, done);
        return check_launch();
    }
    const XGeom &g = pb.ax.gxr32;
    const RSlice rs = rslice(pb, g.L);
    const size_t off = (tile_lds(AX_X, g, sizeof(float)) + 15) / 16 * 16;
    const size_t sh = resid_xfwd_lds(pb, g);
    if (sh > kResidLdsMax) return CANS_ERR_UNSUPPORTED;
    const dim3 grid((unsigned)rslice_blocks(pb, rs));
    if (exact_rows(pb)) {
        CANS_KIND_SWITCH(pb.ax.kind,
            hipLaunchKernelGGL((k_resid_xfwd<KD, true>), grid, dim3(kThreads), sh, s, f, p, out, rs.H, rs.bpp, g,
                               (int)off, pb.ax.d_tw32, lapargs(pb), pb.d_dzf, w.info, w.partials, done));
    } else {
        CANS_KIND_SWITCH(pb.ax.kind,
            hipLaunchKernelGGL((k_resid_xfwd<KD, false>), grid, dim3(kThreads), sh, s, f, p, out, rs.H, rs.bpp, g,
                               (int)off, pb.ax.d_tw32, lapargs(pb), pb.d_dzf, w.info, w.partials, done));
    }
    return check_launch();
}

int launch_resid_norm(const Problem &pb, const Work &w, const double *f, const double *p, const int *done,
                      hipStream_t s)
{
    const RSlice rs = rslice(pb, norm_rows(pb));
    const size_t sh = (size_t)kRowsD * sizeof(double);
    if (exact_rows(pb))
        hipLaunchKernelGGL(k_resid_norm<true>, dim3((unsigned)rslice_blocks(pb, rs)), dim3(kThreads), sh, s, f, p,
                           rs.H, rs.bpp, rs.L, lapargs(pb), pb.d_dzf, w.info, w.partials, done);
    else
        hipLaunchKernelGGL(k_resid_norm<false>, dim3((unsigned)rslice_blocks(pb, rs)), dim3(kThreads), sh, s, f, p,
                           rs.H, rs.bpp, rs.L, lapargs(pb), pb.d_dzf, w.info, w.partials, done);
    return check_launch();
}

// LDS of the residual+transform kernel for x tile geometry g: the FP32
// transform tile, then the FP64 rows
size_t resid_xfwd_lds(const Problem &pb, const XGeom &g)
{
    return (tile_lds(AX_X, g, sizeof(float)) + 15) / 16 * 16 + (size_t)kRowsD * sizeof(double);
}

// dynamic LDS beyond the default 64 KiB for the residual kernels: up to the
// 160 KiB of a CU less each kernel's static LDS (its reductions)
int plan_resid(const Problem &pb)
{
    const void *ks[] = {
#define CANS_RX(K) (const void *)k_resid_xfwd<K, true>, (const void *)k_resid_xfwd<K, false>, \
                   (const void *)k_resid_xfwd_grp<K, true>, (const void *)k_resid_xfwd_grp<K, false>
        CANS_RX(K_P), CANS_RX(K_NN), CANS_RX(K_DD), CANS_RX(K_ND), CANS_RX(K_DN),
        CANS_RX(K_S1), CANS_RX(K_C1), CANS_RX(K_FDN), CANS_RX(K_FND),
#undef CANS_RX
        (const void *)k_resid_norm<true>, (const void *)k_resid_norm<false>,
        (const void *)k_resid_norm_grp<true>, (const void *)k_resid_norm_grp<false>};
    (void)pb;
    for (const void *k : ks) {
        hipFuncAttributes fa;
        if (hipFuncGetAttributes(&fa, k) != hipSuccess) return CANS_ERR_HIP;
        const int dyn = (int)(kResidLdsMax - fa.sharedSizeBytes);
        if (hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, dyn) != hipSuccess) return CANS_ERR_HIP;
    }
    return CANS_OK;
}

// Up to kDirectReduce block partials the last-level kernel reads them
// directly (one launch per check instead of two; small problems are
// launch-bound).

int launch_finalize(const Problem &pb, const Work &w, int nblk, int check, int max_iter, double tol, hipStream_t s)
{
    const double inv_wvol = 1.0 / (pb.wsum * pb.nx * pb.ny);
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

// ---- grouped residual passes and reductions of a batch ---------------------
RJob rjob_xfwd(const Problem &pb, const Work &w, const double *f, const double *p, float *out, const int *done,
               size_t &lds)
{
    const XGeom &g = pb.ax.gxr32;
    const RSlice rs = rslice(pb, g.L);
    lds = resid_xfwd_lds(pb, g);
    RJob j{};
    j.f = f;
    j.p = p;
    j.out = out;
    j.tw = pb.ax.d_tw32;
    j.dzf = pb.d_dzf;
    j.info = w.info;
    j.partials = w.partials;
    j.done = done;
    j.H = rs.H;
    j.bpp = rs.bpp;
    j.L = rs.L;
    j.rows_off = (int)((tile_lds(AX_X, g, sizeof(float)) + 15) / 16 * 16);
    j.nblk = (unsigned)rslice_blocks(pb, rs);
    j.la = lapargs(pb);
    j.g = g;
    return j;
}

RJob rjob_norm(const Problem &pb, const Work &w, const double *f, const double *p, const int *done, size_t &lds)
{
    const RSlice rs = rslice(pb, norm_rows(pb));
    lds = (size_t)kRowsD * sizeof(double);
    RJob j{};
    j.f = f;
    j.p = p;
    j.dzf = pb.d_dzf;
    j.info = w.info;
    j.partials = w.partials;
    j.done = done;
    j.H = rs.H;
    j.bpp = rs.bpp;
    j.L = rs.L;
    j.nblk = (unsigned)rslice_blocks(pb, rs);
    j.la = lapargs(pb);
    return j;
}

// group keys: 2 kind + exact (fused pass), exact (norm pass)
int launch_resid_xfwd_grp(const GroupLaunch &gl, hipStream_t s)
{
    const RJob *j = static_cast<const RJob *>(gl.jobs);
    if (gl.key & 1) {
        CANS_KIND_SWITCH(gl.key >> 1, hipLaunchKernelGGL((k_resid_xfwd_grp<KD, true>), dim3(gl.blocks),
                                                         dim3(kThreads), gl.lds, s, j, gl.start, gl.np));
    } else {
        CANS_KIND_SWITCH(gl.key >> 1, hipLaunchKernelGGL((k_resid_xfwd_grp<KD, false>), dim3(gl.blocks),
                                                         dim3(kThreads), gl.lds, s, j, gl.start, gl.np));
    }
    return check_launch();
}

int launch_resid_norm_grp(const GroupLaunch &gl, hipStream_t s)
{
    const RJob *j = static_cast<const RJob *>(gl.jobs);
    if (gl.key)
        hipLaunchKernelGGL(k_resid_norm_grp<true>, dim3(gl.blocks), dim3(kThreads), gl.lds, s, j, gl.start, gl.np);
    else
        hipLaunchKernelGGL(k_resid_norm_grp<false>, dim3(gl.blocks), dim3(kThreads), gl.lds, s, j, gl.start, gl.np);
    return check_launch();
}

int resid_group_key(const Problem &pb, bool fused) { return fused ? 2 * pb.ax.kind + exact_rows(pb) : exact_rows(pb); }

int launch_reset_grp(const FJob *jobs, int np, hipStream_t s)
{
    hipLaunchKernelGGL(k_reset_grp, dim3(np), dim3(64), 0, s, jobs);
    return check_launch();
}

int launch_mean_rhs_grp(const FJob *jobs, int np, hipStream_t s)
{
    hipLaunchKernelGGL(k_mean_rhs_grp, dim3(np), dim3(kThreads), 0, s, jobs);
    return check_launch();
}

int launch_finalize_grp(const FJob *jobs, int np, int which, int check, int max_iter, double tol, hipStream_t s)
{
    hipLaunchKernelGGL(k_finalize_grp, dim3(np), dim3(kThreads), 0, s, jobs, which, check, max_iter, tol);
    return check_launch();
}
}  // namespace cans

// k_zsolve.hip -- the FP64 z solve of the column systems of eq. (poi_reduced) (Section 2) and
// its launchers.
#include "kcommon.h"

#include <algorithm>
#include <cstdint>

namespace cans {

template <typename T>
__global__ __launch_bounds__(256) void k_zsolve(T *data, ZArgs a, const int *__restrict__ done)
{
    if (done && *done) return;
    const size_t col = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (col >= (size_t)a.nx * a.ny) return;
    zsolve_column(col, data, a);
}

static ZArgs zargs(const Problem &pb, const Work &w, double *removed);

// Partitioned column solve: CPB adjacent columns per block (64 or 32), z split
// into S segments of at most MMAX levels held in registers; a wave holds
// 64/CPB segments of the same columns (see zsolve_core.h).  The body solves
// G column groups of block `blk` (groups blk G .. blk G + G - 1), each with S
// segments: wave w takes segment w % S of group w / S when a wave holds one
// segment (CPB = 64); with two segments a wave (CPB = 32) G is 1.  A grouped
// launch sizes its blocks for its deepest problem, so a shallower one puts
// several column groups in a block; waves beyond G S only take part in the
// barriers.
template <typename T, int MMAX, int CPB, bool FULL, bool CYC, bool PAD>
__device__ __forceinline__ void zsolve_part_body(T *data, const ZArgs &ag, const int *__restrict__ done,
                                                 unsigned blk, int S, int G)
{
    if (done && *done) return;
    constexpr int NQ = CYC ? 8 : 6;  // interface coefficients per segment
    constexpr int GMAX = CYC ? 4 : 16;  // column groups a block (4 x 64 column ends for the periodic form)
    __shared__ double coef[NQ * 1024];
    __shared__ double zabc[3 * 512];  // the z coefficients, staged once per block
    __shared__ double ends[CYC ? 4 * 64 * GMAX : 1];  // CYC: first/last values per column
    constexpr int SPW = 64 / CPB;  // segments per wave
    // PAD: S * MMAX levels (<= 512 for every launched shape), padding rows
    // beyond nz
    const int nzp = PAD ? S * MMAX : ag.nz;
    for (int i = threadIdx.x; i < nzp; i += blockDim.x)
        zpad_row(ag, i, zabc[i], zabc[512 + i], zabc[1024 + i]);
    ZArgs a = ag;
    a.za = zabc;
    a.zb = zabc + 512;
    a.zc = zabc + 1024;
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
    const int gi = SPW == 1 ? w / S : 0;                             // column group of the wave
    const int c = lane % CPB, seg = SPW == 1 ? w - gi * S : w * SPW + lane / CPB;
    const bool act = gi < G && seg < S;
    auto C = [&](int q, int s) -> double & { return coef[q * 1024 + (gi * S + s) * CPB + c]; };
    const size_t col = ((size_t)blk * G + gi) * CPB + c;
    const ZSeg sg = zseg(nzp, S, act ? seg : 0);
    ZLane<MMAX, CYC> L;
    if (act) {
        zp_load<MMAX, FULL, PAD>(L, data, a, col, sg);
        double out[NQ];
        zp_reduce<MMAX, FULL>(L, a, sg, out);
#pragma unroll
        for (int q = 0; q < NQ; ++q) C(q, seg) = out[q];
    }
    __syncthreads();
    if (act && seg == 0 && lane < CPB) {  // the first wave of each group
        zp_interface<CYC>(
            S, [&](int s, int q) -> double & { return C(q, s); }, [&](int s) -> double & { return C(4, s); },
            [&](int s) -> double & { return C(5, s); }, [&](int s) -> double & { return C(6, s); },
            [&](int s) -> double & { return C(7, s); });
    }
    __syncthreads();
    const double xL = act && seg > 0 ? C(5, seg - 1) : 0.0;
    const double xR = act && seg < S - 1 ? C(4, seg + 1) : 0.0;
    if constexpr (CYC) {
        const double xL2 = act && seg > 0 ? C(7, seg - 1) : 0.0;
        const double xR2 = act && seg < S - 1 ? C(6, seg + 1) : 0.0;
        double *E = ends + gi * 4 * 64;
        if (act) {
            zp_finish<MMAX, FULL>(L, a, sg, xL, xR, xL2, xR2);
            // Sherman-Morrison: the column's first and last values of A'^-1 f
            // and A'^-1 u come from its first and last segment
            double y0, z0, yl, zl;
            zp_ends<MMAX, FULL>(L, sg, &y0, &z0, &yl, &zl);
            if (seg == 0) { E[c] = y0; E[64 + c] = z0; }
            if (seg == S - 1) { E[128 + c] = yl; E[192 + c] = zl; }
        }
        __syncthreads();
        if (act) zp_sherman_morrison<MMAX, FULL>(L, a, sg, E[c], E[64 + c], E[128 + c], E[192 + c]);
    } else {
        if (act) zp_finish<MMAX, FULL>(L, a, sg, xL, xR);
    }
    if (act) zp_store<MMAX, FULL, PAD>(L, data, a, col, sg);
    if (a.singular && blk == 0) {
        // the singular column, left out above: projected rhs, pinned last
        // row, zero weighted mean, by one thread with coef as workspace
        __syncthreads();
        if (threadIdx.x == 0) zsolve_singular_ws<T>(0, data, a, coef, coef + 512, 1);
    }
}

template <typename T, int MMAX, int CPB, int NTMAX, bool FULL, bool CYC, bool PAD = false>
__global__ __launch_bounds__(NTMAX) void k_zsolve_part(T *data, ZArgs ag, const int *__restrict__ done)
{
    zsolve_part_body<T, MMAX, CPB, FULL, CYC, PAD>(data, ag, done, blockIdx.x, (int)(blockDim.x >> 6) * (64 / CPB),
                                                   1);
}

template <typename T, int MMAX, int CPB, int NTMAX, bool FULL, bool CYC, bool PAD>
__global__ __launch_bounds__(NTMAX) void k_zsolve_part_grp(const ZJob *__restrict__ jobs,
                                                           const unsigned *__restrict__ start, int np)
{
    const int q = group_find(start, np, blockIdx.x);
    const ZJob &j = jobs[q];
    const unsigned blk = blockIdx.x - start[q];
    if (blk >= j.nblk) return;
    zsolve_part_body<T, MMAX, CPB, FULL, CYC, PAD>(static_cast<T *>(j.data), j.a, j.done, blk, j.S, j.G);
}

// ---------------------------------------------------------------------------
// Persistent, software-pipelined form of the partitioned solve (non-periodic
// z).  A block stays resident and walks tiles of kPipeCols adjacent columns x
// all levels.  The tile is brought into LDS by direct global->LDS loads
// (global_load_lds_dwordx4: the data goes to LDS without passing through
// registers), so the next tile's fetch is in flight while the current one is
// solved.  Per tile: each lane (one column, one segment of MMAX levels) runs
// the single-sweep reduction (zp_sweep_reduce), wave 0 solves the interface
// system of every column from both ends (pipe_interface), each lane finishes its
// segment and stores it.
// DB (two tile buffers): the next fetch starts at the top of an iteration and
// the rhs is read from LDS in the reduction and again in the finish.  !DB (one
// buffer): the rhs is copied to registers first and the next fetch starts
// after that.  lambda of the next tile is loaded after the stores, so the only
// wait for global memory is the one at the top of an iteration.  The barriers
// inside an iteration order LDS traffic only (pipe_lds_barrier): a full
// __syncthreads there would also wait for the next tile's fetch, which writes
// LDS under the vector memory counter.  The next tile is claimed after the
// stores for the same reason: reading the atomic's result waits for every
// vector memory operation issued before it.
// Levels beyond nz (the segments cover S * MMAX >= nz) are the decoupled
// padding rows of zpad_row; their loads are clamped to a real level and
// replaced by zero, their stores skipped.

typedef __attribute__((address_space(3))) void lds_void;

// Workgroup barrier for LDS data: waits for this wave's LDS operations only,
// not for its vector memory operations (global loads into LDS still in flight
// target the other tile buffer).  The memory clobber keeps the compiler from
// moving memory accesses across it.
__device__ __forceinline__ void pipe_lds_barrier()
{
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// The interface system of the pipelined solve in one layout for both roles.
// Wave 0 solves it: lane L < 32 takes the top role of column L (segments 0,
// 1, .. S/2-1), lane L + 32 the bottom role of the same column (segments S-1,
// S-2, .. S/2), as zp_ends_forward / zp_ends_backward do, with the same
// arithmetic.  Step i of a lane's role sits at R[(6 i + q) 64] (R = coef + L):
// a segment of the lower half stores its coefficients (A,B,C,D,E,F) there in
// order, one of the upper half in the bottom role's order (E,C,B,F,A,D), so
// every access is the lane's base plus a constant offset.  Results: slot 4
// of step i takes the unknown next to the role's start (u_s for the top role,
// v_s for the bottom one), slot 5 the other.
constexpr int kPipeRow = 2 * kPipeCols;  // doubles per coefficient row (both roles)
constexpr int kPipeRole[6] = {4, 2, 1, 5, 0, 3};

template <int NB>
__device__ __forceinline__ void pipe_interface(double *R, int n)
{
    auto at = [&](int i, int q) -> double & { return R[(6 * i + q) * kPipeRow]; };
    double y2p = 0, g2p = 0;
#pragma unroll 1
    for (int b0 = 0; b0 < n; b0 += NB) {
        double A[NB], B[NB], Cc[NB], D[NB], E[NB], F[NB];
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            const int i = b0 + j < n ? b0 + j : n - 1;
            A[j] = at(i, 0); B[j] = at(i, 1); Cc[j] = at(i, 2);
            D[j] = at(i, 3); E[j] = at(i, 4); F[j] = at(i, 5);
        }
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            const int i = b0 + j;
            if (i < n) {
                const double inv = rcp64(1.0 - A[j] * g2p);
                const double y1 = (D[j] - A[j] * y2p) * inv;
                const double cg = Cc[j] * g2p;
                const double y2 = (F[j] - Cc[j] * y2p) + cg * y1;
                const double g1 = B[j] * inv;
                const double g2 = E[j] + cg * g1;
                at(i, 0) = y1;
                at(i, 1) = y2;
                at(i, 2) = g1;
                at(i, 3) = g2;
                g2p = g2;
                y2p = y2;
            }
        }
    }
    const double y2o = __shfl_xor(y2p, 32, 64), g2o = __shfl_xor(g2p, 32, 64);
    double prev = zp_ends_meet(y2p, g2p, y2o, g2o);
#pragma unroll 1
    for (int b0 = 0; b0 < n; b0 += NB) {
        double Y1[NB], Y2[NB], G1[NB], G2[NB];
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            const int i0 = n - 1 - (b0 + j);
            const int i = i0 >= 0 ? i0 : 0;
            Y1[j] = at(i, 0); Y2[j] = at(i, 1); G1[j] = at(i, 2); G2[j] = at(i, 3);
        }
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            const int i = n - 1 - (b0 + j);
            if (i >= 0) {
                const double o1 = Y1[j] - G1[j] * prev;
                const double o2 = Y2[j] - G2[j] * prev;
                at(i, 4) = o1;
                at(i, 5) = o2;
                prev = o1;
            }
        }
    }
}

template <typename T>
struct PipeGeom {
    static constexpr int ROW_B = kPipeCols * (int)sizeof(T);  // bytes of one level of a tile
    static constexpr int RPI = 1024 / ROW_B;                    // levels per wave-wide 16-byte load
    static constexpr int GRP_B = 1024 + 64;                     // LDS bytes per load group (padded)
};

template <typename T, int MMAX, bool DB>
__global__ __launch_bounds__(kPipeThreads) void k_zsolve_pipe(T *data, ZArgs ag, int ntiles, unsigned *ctr,
                                                              const int *__restrict__ done)
{
    if (done && *done) return;
    using G = PipeGeom<T>;
    static_assert(MMAX % G::RPI == 0, "segments start on a load group");
    extern __shared__ __align__(16) unsigned char sm[];
    constexpr int SPW = 64 / kPipeCols;              // segments per wave
    const int nw = (int)(blockDim.x >> 6);
    const int S = nw * SPW;                          // segments per column
    const int nzp = S * MMAX;                        // levels incl. padding
    const int nz = ag.nz;
    const int ngrp = nzp / G::RPI;
    const size_t tb = (size_t)ngrp * G::GRP_B;
    unsigned char *buf0 = sm, *buf1 = sm + (DB ? tb : 0);
    double *coef = reinterpret_cast<double *>(sm + (DB ? 2 : 1) * tb);
    double *zabc = coef + 6 * S * kPipeCols;
    // tile numbers from thread 0: [2] the first, [it & 1] the next one in
    // iteration it (two slots, so a slot is rewritten only after a barrier
    // that every thread passes after reading it)
    int *tslot = reinterpret_cast<int *>(zabc + 3 * nzp);
    for (int i = threadIdx.x; i < nzp; i += blockDim.x) zpad_row(ag, i, zabc[i], zabc[nzp + i], zabc[2 * nzp + i]);
    // levels beyond nz are never fetched: their LDS rows stay zero, the
    // padding rows' zero right-hand side
    for (int b = 0; b < (DB ? 2 : 1); ++b)
        for (int e = threadIdx.x; e < (nzp - nz) * kPipeCols; e += blockDim.x) {
            const int k = nz + e / kPipeCols;
            *reinterpret_cast<T *>((b ? buf1 : buf0) + (k / G::RPI) * G::GRP_B + (k % G::RPI) * G::ROW_B +
                                   (e % kPipeCols) * (int)sizeof(T)) = T(0);
        }
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int c = lane % kPipeCols, seg = w * SPW + lane / kPipeCols;
    const int k0 = seg * MMAX;
    const double *za = zabc + k0, *zb = zabc + nzp + k0, *zc = zabc + 2 * nzp + k0;
    const size_t plane = (size_t)ag.nx * ag.ny;
    // the six coefficients of a segment sit kPipeCols doubles apart, so one
    // base address per segment and column serves all of them
    // this lane's slot of the interface layout (pipe_interface), and where
    // the unknowns beside its segment land: v of segment seg-1, u of seg+1
    const int half = S / 2;
    const bool upper = seg >= half;
    double *cme = coef + (upper ? S - 1 - seg : seg) * 6 * kPipeRow + c + (upper ? kPipeCols : 0);
    auto unk = [&](int s2, bool want_v) -> const double & {
        const bool up = s2 >= half;
        return coef[((up ? S - 1 - s2 : s2) * 6 + (up == want_v ? 4 : 5)) * kPipeRow + c + (up ? kPipeCols : 0)];
    };
    // global->LDS: lane = (level in the group, 16-byte chunk of the level)
    constexpr int CHUNK = 16 / (int)sizeof(T);
    const int lrow = lane / (64 / G::RPI);
    const int lcol = (lane % (64 / G::RPI)) * CHUNK;
    auto fetch = [&](int t, unsigned char *buf) {
        size_t c0 = (size_t)t * kPipeCols + lcol;
        if (c0 >= plane) c0 = plane - CHUNK;  // beyond the last column: any real chunk (not used)
        for (int gi = w; gi < ngrp; gi += nw) {
            const int row = gi * G::RPI + lrow;
            if (row < nz)
                __builtin_amdgcn_global_load_lds((const void *)(data + c0 + plane * row),
                                                 (lds_void *)(buf + gi * G::GRP_B), 16, 0, 0);
        }
    };
    const int boff = (k0 / G::RPI) * G::GRP_B + c * (int)sizeof(T);
    auto raw = [&](const unsigned char *buf, int q) -> T {
        return *reinterpret_cast<const T *>(buf + boff + (q / G::RPI) * G::GRP_B + (q % G::RPI) * G::ROW_B);
    };
    const double scale = ag.scale;
    // the singular column (column 0 of a singular problem) is solved apart
    const size_t skip = ag.singular ? 0 : ~(size_t)0;
    const unsigned nxu = (unsigned)ag.nx;
    double lxn = 0, lyn = 0;
    // columns not solved here (beyond the plane, the singular one) get the
    // regular lambda -1
    auto lamload = [&](int t) {
        const size_t col = (size_t)t * kPipeCols + c;
        const bool own = col < plane && col != skip;
        const unsigned cu = own ? (unsigned)col : 0u;
        lxn = own ? ag.lamx[cu % nxu] : -1.0;
        lyn = own ? ag.lamy[cu / nxu] : 0.0;
    };
    // Tiles are claimed from a counter (ctr[0]) by thread 0, two ahead of the
    // one being solved, so a block that starts late (block 0 with the singular
    // column) simply solves fewer.  The last block to finish (ctr[1]) resets
    // both counters for the next launch.
    if (threadIdx.x == 0) tslot[2] = (int)atomicAdd(&ctr[0], 1u);
    __syncthreads();
    int t = tslot[2], it = 0;
    if (t < ntiles) {
        fetch(t, buf0);
        lamload(t);
    }
    int claim = 0;  // thread 0: the tile after the next
    if (threadIdx.x == 0) claim = (int)atomicAdd(&ctr[0], 1u);
    if (ag.singular && blockIdx.x == 0) {
        // the singular column: projected rhs, pinned last row, zero weighted
        // mean, by one thread on a copy staged in the coefficient area
        T *colv = reinterpret_cast<T *>(coef);
        double *wdz = coef + nz, *wc = coef + 2 * nz, *wd = coef + 3 * nz;
        for (int k = threadIdx.x; k < nz; k += blockDim.x) {
            colv[k] = data[plane * k];
            wdz[k] = ag.dzf[k];
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            ZArgs a = ag;
            a.nx = 1;
            a.ny = 1;
            a.za = zabc;
            a.zb = zabc + nzp;
            a.zc = zabc + 2 * nzp;
            a.dzf = wdz;
            zsolve_singular_ws<T>(0, colv, a, wc, wd, 1);
        }
        __syncthreads();
        for (int k = threadIdx.x; k < nz; k += blockDim.x) data[plane * k] = colv[k];
    }
    while (t < ntiles) {
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        if (threadIdx.x == 0) tslot[it & 1] = claim;
        __syncthreads();
        const int tn = tslot[it & 1];
        const unsigned char *cur = (DB && (it & 1)) ? buf1 : buf0;
        const double lam = lxn + lyn;
        T f[DB ? 1 : MMAX];  // !DB: the tile's rhs, as stored
        if constexpr (DB) {
            if (tn < ntiles) fetch(tn, (it & 1) ? buf0 : buf1);
        } else {
#pragma unroll
            for (int q = 0; q < MMAX; ++q) f[q] = raw(cur, q);
            pipe_lds_barrier();
            if (tn < ntiles) fetch(tn, buf0);
        }
        auto fv = [&](int q) -> double {
            if constexpr (DB) return scale * (double)raw(cur, q);
            else return scale * (double)f[q];
        };
        double r[MMAX], out[6];
        zp_sweep_reduce<MMAX>(fv, za, zb, zc, lam, r, out);
#pragma unroll
        for (int q = 0; q < 6; ++q) cme[q * kPipeRow] = upper ? out[kPipeRole[q]] : out[q];
        pipe_lds_barrier();
        if (w == 0) pipe_interface<4>(coef + lane, half);
        pipe_lds_barrier();
        const double xL = seg > 0 ? unk(seg - 1, true) : 0.0;
        const double xR = seg < S - 1 ? unk(seg + 1, false) : 0.0;
        double x[MMAX];
        zp_sweep_finish<MMAX>(fv, za, zc, r, xL, xR, x);
        const size_t col = (size_t)t * kPipeCols + c;
        if (col < plane && col != skip) {
            // levels of this segment below nz; opaque to the compiler so the
            // comparisons are not hoisted out of the tile loop
            int lim = nz - k0;
            asm volatile("" : "+v"(lim));
            T *ptr = data + col + plane * k0;
#pragma unroll
            for (int q = 0; q < MMAX; ++q) {
                if (q < lim) ptr[0] = (T)x[q];
                ptr += plane;
            }
        }
        if (threadIdx.x == 0 && tn < ntiles) claim = (int)atomicAdd(&ctr[0], 1u);
        if (tn < ntiles) lamload(tn);
        t = tn;
        ++it;
    }
    if (threadIdx.x == 0) {
        __threadfence();
        if (atomicAdd(&ctr[1], 1u) == gridDim.x - 1) {
            ctr[0] = 0;
            ctr[1] = 0;
        }
    }
}

// LDS bytes of k_zsolve_pipe for S segments of MMAX levels
template <typename T>
static size_t pipe_lds(int S, int mmax, bool db)
{
    using G = PipeGeom<T>;
    const int nzp = S * mmax;
    return (db ? 2 : 1) * (size_t)(nzp / G::RPI) * G::GRP_B + (size_t)6 * S * kPipeCols * 8 + (size_t)3 * nzp * 8 +
           16;
}

template <typename T>
static const void *pipe_kernel(bool db)
{
    return db ? (const void *)k_zsolve_pipe<T, 16, true> : (const void *)k_zsolve_pipe<T, 16, false>;
}

// Shape of the pipelined solve for this problem (or none): non-periodic z
// with 128 < nz <= 384, 16-level segments, two per wave (S even, <= 24, so
// at most 768 threads and 168 registers a lane).  Two tile buffers when they
// fit the 160 KiB of LDS, else one; 16-byte aligned data.  The grid is one
// resident block per available slot.
template <typename T>
static PipePlan pipe_plan_of(const Problem &pb)
{
    PipePlan pp;
    if (pb.cyclic || pb.nz <= 128 || pb.nz > 384) return pp;
    int S = (pb.nz + 15) / 16;
    S += S & 1;
    const size_t kLds = 160 * 1024;
    const bool db = pipe_lds<T>(S, 16, true) <= kLds;
    const size_t lds = pipe_lds<T>(S, 16, db);
    if (lds > kLds) return pp;
    const void *k = pipe_kernel<T>(db);
    int dev = 0, ncu = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return pp;
    if (hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess) return pp;
    const int threads = 32 * S;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k, threads, lds) != hipSuccess || per < 1) return pp;
    const size_t plane = (size_t)pb.nx * pb.ny;
    const long ntiles = (long)((plane + kPipeCols - 1) / kPipeCols);
    pp.on = true;
    pp.db = db;
    pp.threads = threads;
    pp.lds = lds;
    pp.ntiles = (int)ntiles;
    pp.grid = (int)std::min<long>(ntiles, (long)ncu * per);
    return pp;
}

int plan_zpipe(Problem &pb)
{
    pb.zpipe32 = pipe_plan_of<float>(pb);
    pb.zpipe64 = pipe_plan_of<double>(pb);
    return CANS_OK;
}

template <typename T>
static int launch_zpipe(const Problem &pb, const PipePlan &pp, unsigned *ctr, T *data, double *removed,
                        const int *done, hipStream_t s)
{
    ZArgs za = zargs(pb, Work{}, removed);
    if (pp.db)
        hipLaunchKernelGGL((k_zsolve_pipe<T, 16, true>), dim3(pp.grid), dim3(pp.threads), pp.lds, s, data, za,
                           pp.ntiles, ctr, done);
    else
        hipLaunchKernelGGL((k_zsolve_pipe<T, 16, false>), dim3(pp.grid), dim3(pp.threads), pp.lds, s, data, za,
                           pp.ntiles, ctr, done);
    return check_launch();
}

template <typename T>
static int launch_zsolve(const Problem &pb, const Work &w, T *data, double *removed, const int *done, hipStream_t s)
{
    const PipePlan &pp = sizeof(T) == 4 ? pb.zpipe32 : pb.zpipe64;
    if (pp.on && w.zctr && ((uintptr_t)data & 15) == 0) return launch_zpipe<T>(pb, pp, w.zctr, data, removed, done, s);
    const size_t plane = (size_t)pb.nx * pb.ny;
    const ZPart zp = zpart_shape(pb.nz, pb.cyclic != 0);
    ZArgs za = zargs(pb, w, removed);
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

static ZArgs zargs(const Problem &pb, const Work &w, double *removed)
{
    ZArgs a;
    a.nx = pb.nx; a.ny = pb.ny; a.nz = pb.nz;
    a.za = pb.d_za; a.zb = pb.d_zb; a.zc = pb.d_zc;
    a.lamx = pb.ax.d_lam; a.lamy = pb.ay.d_lam;
    a.dzf = pb.d_dzf; a.wsum = pb.wsum; a.scale = pb.scale;
    a.cyclic = pb.cyclic; a.singular = pb.singular;
    a.wc = w.wc; a.wd = w.wd; a.wz = w.wz;
    a.removed = removed;
    return a;
}

int launch_zsolve_f64(const Problem &pb, const Work &w, double *data, double *removed, hipStream_t s)
{
    return launch_zsolve<double>(pb, w, data, removed, nullptr, s);
}

int launch_zsolve_32(const Problem &pb, const Work &w, float *data, double *removed, const int *done, hipStream_t s)
{
    return launch_zsolve<float>(pb, w, data, removed, done, s);
}

// ---------------------------------------------------------------------------
// Grouped z solves: problems whose partitioned solve takes the same kernel
// variant (segment depth, columns per block, thread bound, full / padded
// segments, periodic or not) share one launch; the launch's blocks hold the
// waves of its deepest member, and a member of S segments puts G = waves / S
// column groups in each of its blocks (CPB = 64; at most 4 periodic).
// Variant codes:
//   0, 1    periodic, 8-level segments, full / ragged
//   2, 3    8-level segments, full / padded
//   4 .. 7  16-level segments of 64 columns: 768 threads full / padded, 1024 full / padded
//   8 .. 11 the same with 32 columns
ZJob zjob_of(const Problem &pb, const Work &w, void *data, double *removed, const int *done, bool fp32, int &key,
             int &threads, unsigned &nblk)
{
    ZJob j{};
    key = -1;
    const PipePlan &pp = fp32 ? pb.zpipe32 : pb.zpipe64;
    const ZPart zp = zpart_shape(pb.nz, pb.cyclic != 0);
    if (pp.on || zp.mmax == 0) return j;  // the pipelined or the plain solve: launched on its own
    const int S = (zp.threads / 64) * (64 / zp.cpb);
    const bool full = pb.nz == S * zp.mmax;
    const bool small = zp.threads <= 768;
    if (pb.cyclic) key = full ? 0 : 1;
    else if (zp.mmax == 8) key = full ? 2 : 3;
    else key = (zp.cpb == 64 ? 4 : 8) + (small ? 0 : 2) + (full ? 0 : 1);
    threads = zp.threads;
    const size_t plane = (size_t)pb.nx * pb.ny;
    j.data = data;
    j.done = done;
    j.S = S;
    j.G = 1;
    j.ngroups = (unsigned)((plane + zp.cpb - 1) / zp.cpb);
    nblk = j.nblk = j.ngroups;
    j.a = zargs(pb, w, removed);
    return j;
}

template <typename T>
static int launch_zgrp(const GroupLaunch &gl, hipStream_t s)
{
    const ZJob *j = static_cast<const ZJob *>(gl.jobs);
    const dim3 grid(gl.blocks), block(gl.threads);
#define CANS_ZG(MM, CPB, NT, FULLV, CYCV, PADV) \
    hipLaunchKernelGGL((k_zsolve_part_grp<T, MM, CPB, NT, FULLV, CYCV, PADV>), grid, block, 0, s, j, gl.start, gl.np)
    switch (gl.key) {
    case 0: CANS_ZG(8, 64, 1024, true, true, false); break;
    case 1: CANS_ZG(8, 64, 1024, false, true, false); break;
    case 2: CANS_ZG(8, 64, 1024, true, false, false); break;
    case 3: CANS_ZG(8, 64, 1024, true, false, true); break;
    case 4: CANS_ZG(16, 64, 768, true, false, false); break;
    case 5: CANS_ZG(16, 64, 768, true, false, true); break;
    case 6: CANS_ZG(16, 64, 1024, true, false, false); break;
    case 7: CANS_ZG(16, 64, 1024, true, false, true); break;
    case 8: CANS_ZG(16, 32, 768, true, false, false); break;
    case 9: CANS_ZG(16, 32, 768, true, false, true); break;
    case 10: CANS_ZG(16, 32, 1024, true, false, false); break;
    case 11: CANS_ZG(16, 32, 1024, true, false, true); break;
    default: return CANS_ERR_INVALID_ARG;
    }
#undef CANS_ZG
    return check_launch();
}

// column groups a block of `waves` waves gives a member of S segments
int zgroup_share(int key, int waves, int S)
{
    if (key >= 8) return 1;  // two segments a wave (32 columns)
    const int g = waves / S;
    const int cap = key <= 1 ? 4 : 16;
    return g < 1 ? 1 : (g > cap ? cap : g);
}

int launch_zsolve_grp(const GroupLaunch &gl, bool fp32, hipStream_t s)
{
    return fp32 ? launch_zgrp<float>(gl, s) : launch_zgrp<double>(gl, s);
}

}  // namespace cans

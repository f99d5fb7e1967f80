// kcommon.h -- helpers shared by the kernel translation units: block
// reductions with a fixed summation order, the XCD-aware tile order, the z
// level of a line, and small launch helpers.
#pragma once

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
    case K_DN: { constexpr int KD = K_DN; __VA_ARGS__; } break;      \
    case K_S1: { constexpr int KD = K_S1; __VA_ARGS__; } break;      \
    case K_C1: { constexpr int KD = K_C1; __VA_ARGS__; } break;      \
    case K_FDN: { constexpr int KD = K_FDN; __VA_ARGS__; } break;    \
    default: { constexpr int KD = K_FND; __VA_ARGS__; } break;       \
    }

static inline int check_launch()
{
    return hipGetLastError() == hipSuccess ? CANS_OK : CANS_ERR_HIP;
}

// ---------------------------------------------------------------------------
// Deterministic block sum of three doubles (fixed order): result in lane 0.
static __device__ void block_sum3(double &a, double &b, double &c)
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
static __device__ void block_max2(double &a, double &b)
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
static __device__ void put_partial(double *partials, unsigned b, double srr, double sff, double spw, double rmax,
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
static __device__ inline unsigned xcd_remap(unsigned b, unsigned nblk)
{
    const unsigned q = nblk / 8, r = nblk % 8, x = b % 8, i = b / 8;
    return x < r ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

// Problem of block b in a grouped launch (one launch for the same kernel
// over several problems): start[] holds the first block of each problem,
// ascending, each a multiple of 8 so that b % 8 (the XCD of the block) is
// also its local index's.
static __device__ __forceinline__ int group_find(const unsigned *__restrict__ start, int np, unsigned b)
{
    int lo = 0, hi = np - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (start[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// z level of line `line` (rows j + ny*k) inside a tile starting at line0
static __device__ inline int line_level(long line, long line0, int k0, int j0, int ny)
{
    const long d = line - line0;
    return (j0 + d < ny) ? k0 : (int)(line / ny);
}

// blocks of the dense (matrix-core) x kernels
static inline dim3 dense_grid(const Problem &pb)
{
    const long nlines = (long)pb.ny * pb.nz;
    return dim3((unsigned)((nlines + kDenseLines - 1) / kDenseLines));
}

// ---------------------------------------------------------------------------
// launchers
// FP64 operator L_h of eq. (poi) (plus the plan's shift) for the residual
// and pressure-update kernels
static inline LapArgs lapargs(const Problem &pb)
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

static inline size_t tile_lds(int axis, const XGeom &g, size_t elem) { return (size_t)tile_slots(axis, g) * 2 * elem; }

// blocks of the first forward x transform, which also leaves the partial
// weighted sums of the rhs (one triple per block)
static inline int xfwd_blocks(const Problem &pb)
{
    const long nlines = (long)pb.ny * pb.nz;
    const int L = pb.ax.dense ? kDenseLines : pb.ax.gx32[1].L;
    return (int)((nlines + L - 1) / L);
}

}  // namespace cans

// dense_core.h -- the x transform of a tile as a dense matrix product on the
// matrix cores (gfx950 MFMA), for short lines in the FP32 refinement path.
//
// out[l][q] = sum_e W[q][e] in[l][e] for the 32 lines of a block, where W is
// the forward transform T (rows in the same order as the FFT path) or the
// inverse B = s T^{-1}.  FP32 operands are split into bf16 pairs,
// x = hi + lo with hi = bf16(x), lo = bf16(x - hi), and the product is
// accumulated in FP32 as hi*hi + hi*lo + lo*hi.  The pair keeps about 16
// significant bits of x (lo drops what lies beyond bf16's 8), and the dropped
// lo*lo term is of the same order, 2^-16 to 2^-17 relative: some 2^7 times
// FP32's own rounding.  The products are therefore well short of FP32
// accuracy; iterative refinement on the FP64 residual recovers the rest (one
// more correction than the FFT form needs).
//
// Layout of v_mfma_f32_32x32x8 (bf16): lane l holds A[l%32][4(l/32)+i] and
// B[4(l/32)+i][l%32] for i < 4; accumulator r of lane l is
// D[8(r/4) + 4(l/32) + r%4][l%32].
#pragma once

#include <hip/hip_runtime.h>

#include "xform_core.h"

namespace cans {

constexpr int kDenseLines = 32;   // lines per block
constexpr int kDenseMaxN = 512;   // n = 128 .. 512, multiple of 128

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// round-to-nearest-even FP32 -> bf16 bits, and back
CANS_HD unsigned short to_bf16(float x)
{
    unsigned u;
    __builtin_memcpy(&u, &x, 4);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}
CANS_HD float from_bf16(unsigned short h)
{
    const unsigned u = (unsigned)h << 16;
    float x;
    __builtin_memcpy(&x, &u, 4);
    return x;
}

// Row stride of a line in LDS (bf16 elements): n + 4, so that the 32 rows a
// wave reads at one k fall on distinct banks (a stride of n would put them
// all on the same ones).
CANS_HD int dense_ld(int n) { return n + 4; }

// LDS bytes of a dense tile (bf16 hi and lo of 32 lines)
CANS_HD size_t dense_lds(int n) { return (size_t)kDenseLines * dense_ld(n) * 2 * sizeof(unsigned short); }

// Position of W[q][e] in the k-blocked layout of the matrices on the device:
// blocks of 8 consecutive e, each block holding all n rows q with their 8
// values contiguous, so the 64 lanes of an operand load read 512 contiguous
// bytes (32 rows x 2 halves of 4).
CANS_HD size_t dense_wpos(int n, int q, int e) { return ((size_t)(e >> 3) * n + q) * 8 + (e & 7); }

// Whole dense transform of a block: src(e, l) -> put(q, l, v).
// Wh/Wl: bf16 hi/lo of W in the k-blocked layout (dense_wpos).  256 threads;
// wave w computes output columns [w n/4, (w+1) n/4) as NT = n/128 tiles of
// 32, with NT fixed at compile time so the accumulators stay in place, and
// the W operands of step k0 + 8 are loaded while step k0 is multiplied.
template <int NT, typename Src, typename Put>
__device__ void dense_transform_nt(int n, unsigned magn, const Src &src, const Put &put,
                                   const unsigned short *__restrict__ Wh, const unsigned short *__restrict__ Wl,
                                   unsigned short *lds)
{
    const int ld = dense_ld(n);
    unsigned short *Ah = lds, *Al = lds + kDenseLines * ld;
    const int tid = threadIdx.x;
    for (int idx = tid; idx < kDenseLines * n; idx += 256) {
        const int l = (int)udiv((unsigned)idx, (unsigned)n, magn), e = idx - l * n;
        const float a = (float)src(e, l);
        const unsigned short h = to_bf16(a);
        Ah[l * ld + e] = h;
        Al[l * ld + e] = to_bf16(a - from_bf16(h));
    }
    __syncthreads();
    const int lane = tid & 63, w = tid >> 6;
    const int row = lane & 31, kq = 4 * (lane >> 5);
    const int col0 = w * (n / 4);
    f32x16 acc[NT];
#pragma unroll
    for (int c = 0; c < NT; ++c)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[c][r] = 0.f;
    auto fetch = [&](int k0, bf16x4 *h, bf16x4 *lo) {
#pragma unroll
        for (int c = 0; c < NT; ++c) {
            const size_t p = dense_wpos(n, col0 + c * 32 + row, k0 + kq);
            h[c] = *reinterpret_cast<const bf16x4 *>(Wh + p);
            lo[c] = *reinterpret_cast<const bf16x4 *>(Wl + p);
        }
    };
    auto mma = [&](int k0, const bf16x4 *h, const bf16x4 *lo) {
        const bf16x4 ah = *reinterpret_cast<const bf16x4 *>(Ah + row * ld + k0 + kq);
        const bf16x4 al = *reinterpret_cast<const bf16x4 *>(Al + row * ld + k0 + kq);
#pragma unroll
        for (int c = 0; c < NT; ++c) {
            acc[c] = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(ah, h[c], acc[c], 0, 0, 0);
            acc[c] = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(ah, lo[c], acc[c], 0, 0, 0);
            acc[c] = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(al, h[c], acc[c], 0, 0, 0);
        }
    };
    // two operand buffers in turn (n / 8 steps, an even count): the loads of
    // one step are in flight while the other step is multiplied
    bf16x4 h0[NT], l0[NT], h1[NT], l1[NT];
    fetch(0, h0, l0);
    for (int k0 = 0; k0 < n; k0 += 16) {
        fetch(k0 + 8, h1, l1);
        __builtin_amdgcn_sched_barrier(0);
        mma(k0, h0, l0);
        __builtin_amdgcn_sched_barrier(0);
        fetch(k0 + 16 < n ? k0 + 16 : k0, h0, l0);  // last step: a harmless re-read
        __builtin_amdgcn_sched_barrier(0);
        mma(k0 + 8, h1, l1);
        __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int c = 0; c < NT; ++c) {
        const int q = col0 + c * 32 + (lane & 31);
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int l = 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
            put(q, l, acc[c][r]);
        }
    }
}

template <typename Src, typename Put>
__device__ void dense_transform(int n, unsigned magn, const Src &src, const Put &put,
                                const unsigned short *__restrict__ Wh, const unsigned short *__restrict__ Wl,
                                unsigned short *lds)
{
    switch (n >> 7) {  // n = 128 .. 512, a multiple of 128
    case 1: dense_transform_nt<1>(n, magn, src, put, Wh, Wl, lds); break;
    case 2: dense_transform_nt<2>(n, magn, src, put, Wh, Wl, lds); break;
    case 3: dense_transform_nt<3>(n, magn, src, put, Wh, Wl, lds); break;
    default: dense_transform_nt<4>(n, magn, src, put, Wh, Wl, lds); break;
    }
}

}  // namespace cans

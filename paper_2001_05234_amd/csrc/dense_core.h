// dense_core.h -- the x transform of a tile as a dense matrix product on the
// matrix cores (gfx950 MFMA), for short lines in the FP32 refinement path.
//
// out[l][q] = sum_e W[q][e] in[l][e] for the 32 lines of a block, where W is
// the forward transform T (rows in the same order as the FFT path) or the
// inverse B = s T^{-1}.  FP32 operands are split into bf16 pairs,
// x = hi + lo with hi = bf16(x), lo = bf16(x - hi), and the product is
// accumulated in FP32 as hi*hi + hi*lo + lo*hi (the lo*lo term is below FP32
// resolution), giving close to FP32 accuracy at bf16 matrix-core rate.
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

// LDS bytes of a dense tile (bf16 hi and lo of 32 lines of n)
CANS_HD size_t dense_lds(int n) { return (size_t)kDenseLines * n * 2 * sizeof(unsigned short); }

// Whole dense transform of a block: src(e, l) -> put(q, l, v).
// Wh/Wl: bf16 hi/lo of W, row-major [n][n] (row = output q).  256 threads.
template <typename Src, typename Put>
__device__ void dense_transform(int n, unsigned magn, const Src &src, const Put &put,
                                const unsigned short *__restrict__ Wh, const unsigned short *__restrict__ Wl,
                                unsigned short *lds)
{
    unsigned short *Ah = lds, *Al = lds + kDenseLines * n;
    const int tid = threadIdx.x;
    for (int idx = tid; idx < kDenseLines * n; idx += 256) {
        const int l = (int)udiv((unsigned)idx, (unsigned)n, magn), e = idx - l * n;
        const float a = (float)src(e, l);
        const unsigned short h = to_bf16(a);
        Ah[l * n + e] = h;
        Al[l * n + e] = to_bf16(a - from_bf16(h));
    }
    __syncthreads();
    const int lane = tid & 63, w = tid >> 6;
    const int row = lane & 31, kq = 4 * (lane >> 5);
    const int ntile = n / 128;  // 32-column tiles per wave (1..4)
    const int col0 = w * (n / 4);
    f32x16 acc[4];
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[c][r] = 0.f;
    for (int k0 = 0; k0 < n; k0 += 8) {
        const bf16x4 ah = *reinterpret_cast<const bf16x4 *>(Ah + row * n + k0 + kq);
        const bf16x4 al = *reinterpret_cast<const bf16x4 *>(Al + row * n + k0 + kq);
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            if (c < ntile) {
                const size_t wrow = (size_t)(col0 + c * 32 + row) * n + k0 + kq;
                const bf16x4 bh = *reinterpret_cast<const bf16x4 *>(Wh + wrow);
                const bf16x4 bl = *reinterpret_cast<const bf16x4 *>(Wl + wrow);
                acc[c] = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(ah, bh, acc[c], 0, 0, 0);
                acc[c] = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(ah, bl, acc[c], 0, 0, 0);
                acc[c] = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(al, bh, acc[c], 0, 0, 0);
            }
        }
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        if (c < ntile) {
            const int q = col0 + c * 32 + (lane & 31);
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int l = 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                put(q, l, acc[c][r]);
            }
        }
    }
}

}  // namespace cans

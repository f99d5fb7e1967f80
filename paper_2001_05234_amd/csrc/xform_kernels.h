// xform_kernels.h -- the x and y transform kernels (LDS radix FFT) and the
// dense matrix-core x kernel of Section 2's F^x, F^y (eq. (poi_reduced)),
// as templates; each k_*.hip translation unit instantiates the ones its
// launchers use.
#pragma once

#include "kcommon.h"

namespace cans {

// x transform: a block holds L consecutive x lines (rows j + ny*k).
// EPI 0: out = v;  EPI 1: out = out + v - info[I_MEANP] (refinement update).
// `wsum_part` (optional, forward only): block partial sums of dzf_k * in in
// FP64, so the exact weighted mean of the rhs is known in refinement mode.
// At least 4 waves per SIMD: the staged FP64 inverses would otherwise take
// 145 VGPRs and run 3 (the cap costs them a small spill and is faster).
// xform_x_body is the work of block `blk`; the kernels below run it for one
// problem (blk = blockIdx.x) or for a group of problems (grouped launches).
template <int KIND, bool FWD, typename T, typename Tin, typename Tout, int EPI>
__device__ __forceinline__ void xform_x_body(const Tin *in, Tout *out, long nlines, const XGeom &g,
                                             const cx<T> *__restrict__ tw, const double *__restrict__ info,
                                             const int *__restrict__ done, const double *__restrict__ dzf,
                                             int ny, double *__restrict__ wsum_part, unsigned blk)
{
    if (done && *done) return;
    extern __shared__ __align__(16) unsigned char smem[];
    const Tile<AX_X, T> tile{reinterpret_cast<cx<T> *>(smem), g.L, g.RS, g.psh};
    const int n = g.nl;
    const long line0 = (long)blk * g.L;
    const int k0 = (int)(line0 / ny), j0 = (int)(line0 - (long)k0 * ny);
    const double mp = EPI == 1 ? info[I_MEANP] : 0.0;
    // output of line l, real q; two adjacent reals (q even, n even: an
    // aligned pair) in one store
    struct Put {
        Tout *out;
        long line0, nlines;
        int n;
        double mp;
        __device__ void operator()(int q, int l, T v) const
        {
            const long line = line0 + l;
            if (line < nlines) {
                const size_t idx = (size_t)line * n + q;
                if (EPI == 1) out[idx] = (Tout)((double)out[idx] + (double)v - mp);
                else out[idx] = (Tout)v;
            }
        }
        __device__ void operator()(int q, int l, T v0, T v1) const
        {
            const long line = line0 + l;
            if (line < nlines) {
                using V2 = typename std::conditional<sizeof(Tout) == 4, float2, double2>::type;
                V2 *d = reinterpret_cast<V2 *>(out + (size_t)line * n + q);
                V2 w;
                if (EPI == 1) {
                    const V2 o = *d;
                    w.x = (Tout)((double)o.x + (double)v0 - mp);
                    w.y = (Tout)((double)o.y + (double)v1 - mp);
                } else {
                    w.x = (Tout)v0;
                    w.y = (Tout)v1;
                }
                *d = w;
            }
        }
    };
    const Put put{out, line0, nlines, n, mp};
    // The block's lines are staged in LDS first with coalesced loads, every
    // load in flight at once (the syntheses of the inverses and the extended
    // lines of the face-located transforms read each input twice; the forward
    // transforms gain from the wide loads alone).  `acc` collects the partial
    // weighted sum of the input when wsum_part is given.
    double acc = 0;
    if (g.nl == g.n) {
        // the lines are contiguous: each thread loads its pairs of reals (one
        // complex slot each) as vectors
        using V2 = typename std::conditional<sizeof(Tin) == 4, float2, double2>::type;
        constexpr int SP = sizeof(T) == 4 ? 16 : 8;  // slots a thread (tile capacity / kThreads)
        const int M = g.M, P = M * g.L;
        const long left = nlines - line0;
        const int avail = (int)((left < g.L ? left : (long)g.L) * M);
        const V2 *src2 = reinterpret_cast<const V2 *>(in + (size_t)line0 * n);
        // every line of the tile on level k0: plain sums, weighted once
        const bool one_level = j0 + g.L <= ny;
        for (int base = 0; base < P; base += SP * kThreads) {  // one round for the default tiles
            V2 v[SP];
#pragma unroll
            for (int u = 0; u < SP; ++u) {
                const int idx = base + threadIdx.x + u * kThreads;
                v[u] = src2[idx < avail ? idx : avail - 1];
            }
#pragma unroll
            for (int u = 0; u < SP; ++u) {
                const int idx = base + threadIdx.x + u * kThreads;
                if (idx < P) {
                    const int l = (int)udiv((unsigned)idx, (unsigned)M, g.magM), m = idx - l * M;
                    const bool ok = idx < avail;
                    tile.at(m, l) = ok ? mk((T)v[u].x, (T)v[u].y) : mk(T(0), T(0));
                    if (wsum_part && ok) {
                        const double s2 = (double)v[u].x + (double)v[u].y;
                        if (one_level) acc += s2;
                        else acc += dzf[line_level(line0 + l, line0, k0, j0, ny)] * s2;
                    }
                }
            }
        }
        if (wsum_part && one_level) acc *= dzf[k0];
    } else {
        for (int idx = threadIdx.x; idx < n * g.L; idx += kThreads) {
            const int l = (int)udiv((unsigned)idx, (unsigned)n, g.magN), e = idx - l * n;
            const long line = line0 + l;
            const T x = line < nlines ? (T)in[line * n + e] : T(0);
            tile_real(tile, e, l) = x;
            if (wsum_part && line < nlines) acc += dzf[line_level(line, line0, k0, j0, ny)] * (double)in[line * n + e];
        }
    }
    __syncthreads();
    auto src = [&](int e, int l) -> T { return tile_real(tile, e, l); };
    tile_transform<KIND, FWD, AX_X, true, true>(threadIdx.x, kThreads, g, src, put, tile, tile, tw, BlockSync());
    if (wsum_part) {
        double z1 = 0, z2 = 0;
        block_sum3(acc, z1, z2);
        if (threadIdx.x == 0) {
            wsum_part[kNP * blk] = acc;
        }
    }
}

template <int KIND, bool FWD, typename T, typename Tin, typename Tout, int EPI>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(4)))
void k_xform_x(const Tin *in, Tout *out, long nlines, XGeom g, const cx<T> *__restrict__ tw,
               const double *__restrict__ info, const int *__restrict__ done, const double *__restrict__ dzf,
               int ny, double *__restrict__ wsum_part)
{
    xform_x_body<KIND, FWD, T, Tin, Tout, EPI>(in, out, nlines, g, tw, info, done, dzf, ny, wsum_part, blockIdx.x);
}


template <int KIND, bool FWD, typename T, typename Tin, typename Tout, int EPI>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(4)))
void k_xform_x_grp(const XJob *__restrict__ jobs, const unsigned *__restrict__ start, int np)
{
    const int p = group_find(start, np, blockIdx.x);
    const XJob &j = jobs[p];
    const unsigned blk = blockIdx.x - start[p];
    if (blk >= j.nblk) return;
    xform_x_body<KIND, FWD, T, Tin, Tout, EPI>(static_cast<const Tin *>(j.in), static_cast<Tout *>(j.out),
                                               j.nlines, j.g, static_cast<const cx<T> *>(j.tw), j.info, j.done,
                                               j.dzf, j.ny, j.wsum_part, blk);
}

// y transform: tile (t, k) holds columns i0 .. i0+L-1 of plane k, all ny
// rows; each global row segment of L elements is contiguous.  Block `blk` of
// `nblk` (tile order remapped so that each XCD runs a contiguous range).
template <int KIND, bool FWD, typename T, typename Tio>
__device__ __forceinline__ void xform_y_body(const Tio *in, Tio *out, int nx, int ny, int ntx, const XGeom &g,
                                             const cx<T> *__restrict__ tw, const int *__restrict__ done,
                                             unsigned blk, unsigned nblk)
{
    if (done && *done) return;
    extern __shared__ __align__(16) unsigned char smem[];
    const Tile<AX_Y, T> tile{reinterpret_cast<cx<T> *>(smem), g.L, g.RS, g.psh};
    const unsigned t = xcd_remap(blk, nblk);
    const int i0 = (int)(t % ntx) * g.L;
    const size_t base = (size_t)(t / ntx) * nx * ny;
    auto put = [&](int q, int l, T v) {
        const int i = i0 + l;
        if (i < nx) out[base + (size_t)q * nx + i] = (Tio)v;
    };
    constexpr int V = 16 / sizeof(Tio);  // reals of one 16-byte load
    if (reads_twice(KIND, FWD) && g.L % V == 0 && nx % V == 0) {
        // transforms that read each input twice (the syntheses, the extended
        // face lines) stage the tile's row segments in LDS: 16-byte loads,
        // every one in flight before the first LDS write (measured: the
        // forward transforms gain nothing from it and read their rows
        // directly)
        using VT = typename std::conditional<sizeof(Tio) == 4, float4, double2>::type;
        const int vpr = g.L / V;              // vectors of a row segment
        const int nv = g.nl * vpr;            // vectors of the tile
        const int lg = vpr == 1 ? 0 : (vpr == 2 ? 1 : (vpr == 4 ? 2 : (vpr == 8 ? 3 : 4)));
        constexpr int SV = 8;                 // vectors a thread per round (tile capacity / kThreads)
        for (int b0 = 0; b0 < nv; b0 += SV * kThreads) {
            VT v[SV];
#pragma unroll
            for (int u = 0; u < SV; ++u) {
                const int idx = min(b0 + (int)threadIdx.x + u * kThreads, nv - 1);
                const int e = idx >> lg, c = (idx - (e << lg)) * V;
                const int i = min(i0 + c, nx - V);  // a segment past the last column: any in-range load
                v[u] = *reinterpret_cast<const VT *>(in + base + (size_t)e * nx + i);
            }
#pragma unroll
            for (int u = 0; u < SV; ++u) {
                const int idx = b0 + (int)threadIdx.x + u * kThreads;
                if (idx < nv) {
                    const int e = idx >> lg, c = (idx - (e << lg)) * V;
                    const bool in_x = i0 + c < nx;
                    const Tio *w = reinterpret_cast<const Tio *>(&v[u]);
#pragma unroll
                    for (int q = 0; q < V; ++q) tile_real(tile, e, c + q) = in_x ? (T)w[q] : T(0);
                }
            }
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

template <int KIND, bool FWD, typename T, typename Tio>
__global__ __launch_bounds__(kThreads) void k_xform_y(const Tio *in, Tio *out, int nx, int ny, int ntx, XGeom g,
                                                      const cx<T> *__restrict__ tw,
                                                      const int *__restrict__ done)
{
    xform_y_body<KIND, FWD, T, Tio>(in, out, nx, ny, ntx, g, tw, done, blockIdx.x, gridDim.x);
}


template <int KIND, bool FWD, typename T, typename Tio>
__global__ __launch_bounds__(kThreads) void k_xform_y_grp(const YJob *__restrict__ jobs,
                                                          const unsigned *__restrict__ start, int np)
{
    const int p = group_find(start, np, blockIdx.x);
    const YJob &j = jobs[p];
    const unsigned blk = blockIdx.x - start[p];
    if (blk >= j.nblk) return;
    Tio *d = static_cast<Tio *>(j.data);
    xform_y_body<KIND, FWD, T, Tio>(d, d, j.nx, j.ny, j.ntx, j.g, static_cast<const cx<T> *>(j.tw), j.done, blk,
                                    j.nblk);
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

}  // namespace cans

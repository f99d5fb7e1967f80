// tables.h -- host-side tables of the eigenfunction expansion (Section 2):
// the boundary pair of each axis, the FFT radix plan and tile shape, the
// modified wavenumbers mu(q) of each transform row, the transform twiddles,
// and the conservative z coefficients of a stretched z.  Computed in long
// double and rounded once.
#pragma once

#include <algorithm>
#include <cmath>
#include <vector>

#include "../../include/cans_poisson.h"
#include "xform_core.h"

namespace cans {

inline bool face_code(int c) { return c == CANS_BC_DIRICHLET_FACE || c == CANS_BC_NEUMANN_FACE; }

// transform kind of an x or y axis from its two boundary codes, -1 if the
// pair is invalid
inline int axis_kind(int lo, int hi)
{
    if (face_code(lo) || face_code(hi)) {
        if (!face_code(lo) || !face_code(hi)) return -1;
        if (lo == CANS_BC_DIRICHLET_FACE) return hi == CANS_BC_DIRICHLET_FACE ? K_S1 : K_FDN;
        return hi == CANS_BC_NEUMANN_FACE ? K_C1 : K_FND;
    }
    if (lo == CANS_BC_PERIODIC || hi == CANS_BC_PERIODIC)
        return (lo == CANS_BC_PERIODIC && hi == CANS_BC_PERIODIC) ? K_P : -1;
    if (lo == CANS_BC_NEUMANN && hi == CANS_BC_NEUMANN) return K_NN;
    if (lo == CANS_BC_DIRICHLET && hi == CANS_BC_DIRICHLET) return K_DD;
    if (lo == CANS_BC_NEUMANN && hi == CANS_BC_DIRICHLET) return K_ND;
    if (lo == CANS_BC_DIRICHLET && hi == CANS_BC_NEUMANN) return K_DN;
    return -1;
}

// Radix plan of an M-point FFT: radix `rmax` (8 or 4) first, then the
// remaining power of two, then 3s and 5s.  Returns false if M has another
// prime factor.
inline bool factor(int M, XGeom &g, int rmax = 8)
{
    int r = M, nst = 0;
    int rads[kMaxStages];
    if (rmax >= 8)
        while (r % 8 == 0 && nst < kMaxStages) { rads[nst++] = 8; r /= 8; }
    while (r % 4 == 0 && nst < kMaxStages) { rads[nst++] = 4; r /= 4; }
    if (r % 2 == 0 && nst < kMaxStages) { rads[nst++] = 2; r /= 2; }
    while (r % 3 == 0 && nst < kMaxStages) { rads[nst++] = 3; r /= 3; }
    while (r % 5 == 0 && nst < kMaxStages) { rads[nst++] = 5; r /= 5; }
    if (r != 1) return false;
    g.nst = nst;
    int s = 1;
    for (int i = 0; i < nst; ++i) {
        g.rad[i] = rads[i];
        g.str[i] = s;
        g.mag_s[i] = mag_of((unsigned)s);
        g.mag_nb[i] = mag_of((unsigned)(M / rads[i]));
        s *= rads[i];
    }
    return true;
}

inline int pow2floor(long v)
{
    int p = 1;
    while ((long)p * 2 <= v) p *= 2;
    return p;
}

inline bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

// Tile of L lines for an n-point transform with elements of `elem` bytes:
// lines per tile such that a tile holds at most 4096 complex values (2048 in
// FP64), 3840 when M has a factor 3 or 5 (the in-place stages hold at most
// 16 complex values per thread of a 256-thread block); x tiles at most 256
// lines (short lines fill a tile with many), y tiles at most 32 (FP32) / 16
// (FP64) columns.
inline int tile_lines(int axis, int n, int elem)
{
    const int M = n / 2 > 0 ? n / 2 : 1;
    long cap = elem == 8 ? 2048 : 4096;
    if (!is_pow2(M)) cap = std::min<long>(cap, 3840);
    const int lmax = axis == AX_X ? 256 : (elem == 8 ? 16 : 32);
    return std::max(1, std::min(lmax, pow2floor(std::max<long>(1, cap / M))));
}

// bytes of LDS a tile takes
inline size_t tile_bytes(int axis, const XGeom &g, int elem) { return (size_t)tile_slots(axis, g) * 2 * elem; }

// Geometry of the tile of a transform of `kind` over lines of nl reals; L =
// 0 takes the default lines per tile, rmax the radix preference.  False if
// the tile does not fit.
inline bool make_geom(XGeom &g, int axis, int kind, int nl, int elem, int L = 0, int rmax = 8)
{
    const int n = fft_len(kind, nl);
    g = XGeom{};
    if (n < 2 || n % 2) return false;
    g.n = n;
    g.nl = nl;
    g.M = n / 2;
    g.L = L > 0 ? L : tile_lines(axis, n, elem);
    if (!is_pow2(g.L) || g.L > (axis == AX_X ? 256 : 32)) return false;
    g.lgL = 0;
    while ((1 << g.lgL) < g.L) ++g.lgL;
    g.psh = elem == 8 ? 4 : 5;  // 256-byte LDS rows of 16-byte / 8-byte slots
    g.RS = g.M + ((g.M - 1) >> g.psh) + 1;
    g.magM = mag_of((unsigned)g.M);
    g.magN = mag_of((unsigned)g.nl);
    if (!factor(g.M, g, rmax)) return false;
    if (tile_bytes(axis, g, elem) > 65536) return false;
    // every in-place stage must fit the per-thread capacity of a 256-thread block
    for (int st = 0; st < g.nst; ++st)
        if ((long)(g.M / g.rad[st]) * g.L > (long)(kMaxC / g.rad[st]) * 256) return false;
    return true;
}


inline long double mu_row(int kind, int n, int q)
{
    const long double pi = 3.141592653589793238462643383279502884L;
    long double th;
    switch (kind) {
    case K_P: {
        const int l = q == 0 ? 0 : (q == 1 ? n / 2 : q / 2);
        th = pi * l / n;
        break;
    }
    case K_NN: th = pi * q / (2.0L * n); break;
    case K_DD: th = pi * (q + 1) / (2.0L * n); break;
    case K_S1: th = pi * (q + 1) / (2.0L * (n + 1)); break;
    case K_C1: th = pi * q / (2.0L * (n - 1)); break;
    default: th = pi * (2 * q + 1) / (4.0L * n); break;  // ND, DN, FDN, FND
    }
    const long double s = sinl(th);
    return -4.0L * s * s;
}


// Twiddles of an n-point transform (layout in xform_core.h).
inline std::vector<cx<double>> twiddles(int n)
{
    const long double pi = 3.141592653589793238462643383279502884L;
    const int M = n / 2;
    std::vector<cx<double>> t(tw_size(M));
    auto put = [&](int idx, long double ang) { t[idx] = mk((double)cosl(ang), (double)sinl(ang)); };
    for (int j = 0; j < M; ++j) put(tw_fft(M) + j, -2 * pi * j / M);
    for (int k = 0; k < M; ++k) put(tw_split(M) + k, -2 * pi * k / n);
    for (int q = 0; q <= M; ++q) put(tw_qw(M) + q, pi * q / (2.0L * n));
    for (int m = 0; m < M; ++m) put(tw_pre4(M) + m, -pi * (4 * m + 1) / (4.0L * n));
    for (int k = 0; k < M; ++k) put(tw_post4(M) + k, -pi * k / n);
    return t;
}

// mu(q)/h^2 for every row q of an axis
inline std::vector<double> lambdas(int kind, int n, double h)
{
    std::vector<double> lam(n);
    for (int q = 0; q < n; ++q) lam[q] = (double)(mu_row(kind, n, q) / ((long double)h * h));
    return lam;
}

// Kind of the z axis: as axis_kind for the cell-centred pairs, plus a
// face-located field with CANS_BC_DIRICHLET_FACE at both ends, which solves
// as Dirichlet-Dirichlet: neither periodic nor singular.  No other face pair
// on z.
inline int z_kind(int lo, int hi)
{
    if (face_code(lo) || face_code(hi))
        return (lo == CANS_BC_DIRICHLET_FACE && hi == CANS_BC_DIRICHLET_FACE) ? K_DD : -1;
    return axis_kind(lo, hi);
}

// z widths a problem is given: nz cells, or the nz+1 cells whose interior
// faces carry a face-located field
inline int z_widths(int nz, int lo) { return lo == CANS_BC_DIRICHLET_FACE ? nz + 1 : nz; }

// z volume weight of each of the nz unknowns: its cell width, or for a
// face-located field the centre-to-centre span around the face
inline std::vector<double> z_weights(int nz, int lo, const double *dz)
{
    std::vector<double> w(dz, dz + nz);
    if (lo == CANS_BC_DIRICHLET_FACE)
        for (int k = 0; k < nz; ++k) w[k] = (double)(((long double)dz[k] + dz[k + 1]) / 2);
    return w;
}

// Conservative z coefficients of cells 0..nz-1.  Folded (a, b, c): wall
// ghost rules applied to the diagonal, for the tridiagonal solve.  Unfolded
// (af, cf): bare face couplings with ghost spacing at walls, for the
// residual stencil.  A face-located field (lo == hi ==
// CANS_BC_DIRICHLET_FACE) takes the nz+1 widths of its cells in dzf.
inline void zcoef(int nz, int lo, int hi, const std::vector<double> &dzf, std::vector<double> &a,
                  std::vector<double> &b, std::vector<double> &c, std::vector<double> &af,
                  std::vector<double> &cf)
{
    a.assign(nz, 0); b.assign(nz, 0); c.assign(nz, 0); af.assign(nz, 0); cf.assign(nz, 0);
    if (lo == CANS_BC_DIRICHLET_FACE) {
        // unknown k on the face between cells k and k+1: couplings across
        // one cell width, control volume of half of each cell; the wall
        // faces hold zero, so the end rows drop their outer coupling and keep
        // the full diagonal.  The residual stencil applies the antisymmetric
        // ghost at these walls, so its wall couplings af[0], cf[nz-1] are
        // halved: (a/2)(w - (-w)) = a w, exactly the zero wall value.
        for (int k = 0; k < nz; ++k) {
            const long double below = dzf[k], above = dzf[k + 1], cv = (below + above) / 2;
            const long double ak = 1 / (below * cv), ck = 1 / (above * cv);
            af[k] = a[k] = (double)ak;
            cf[k] = c[k] = (double)ck;
            b[k] = (double)-(ak + ck);
        }
        a[0] = 0;
        c[nz - 1] = 0;
        af[0] *= 0.5;
        cf[nz - 1] *= 0.5;
        return;
    }
    for (int k = 0; k < nz; ++k) {
        const long double f = dzf[k];
        long double cm, cp;
        if (k > 0) cm = (dzf[k - 1] + f) / 2;
        else cm = lo == CANS_BC_PERIODIC ? (dzf[nz - 1] + f) / 2 : f;
        if (k < nz - 1) cp = (f + dzf[k + 1]) / 2;
        else cp = hi == CANS_BC_PERIODIC ? (f + dzf[0]) / 2 : f;
        const long double ak = 1 / (cm * f), ck = 1 / (cp * f);
        af[k] = (double)ak;
        cf[k] = (double)ck;
        a[k] = (double)ak;
        c[k] = (double)ck;
        b[k] = (double)-(ak + ck);
    }
    // wall rows: Neumann p_ghost = p, Dirichlet p_ghost = -p
    if (lo == CANS_BC_NEUMANN) { b[0] = (double)((long double)b[0] + af[0]); a[0] = 0; }
    if (lo == CANS_BC_DIRICHLET) { b[0] = (double)((long double)b[0] - af[0]); a[0] = 0; }
    if (hi == CANS_BC_NEUMANN) { b[nz - 1] = (double)((long double)b[nz - 1] + cf[nz - 1]); c[nz - 1] = 0; }
    if (hi == CANS_BC_DIRICHLET) { b[nz - 1] = (double)((long double)b[nz - 1] - cf[nz - 1]); c[nz - 1] = 0; }
}

// normalisation s of B T = s I (n: reals of a line)
inline int xform_scale(int kind, int n)
{
    if (kind == K_S1 || kind == K_C1) return fft_len(kind, n);
    return (kind == K_ND || kind == K_DN) ? n / 2 : n;
}

// face kinds: zero mode of DCT-I (q = 0), as P and NN
inline bool has_zero_mode(int kind) { return kind == K_P || kind == K_NN || kind == K_C1; }

// Row q of the forward transform of an axis as a dense vector (the same rows,
// order and signs the FFT path produces): T[q][e], long double.
inline std::vector<long double> dense_forward(int kind, int n)
{
    const long double pi = 3.141592653589793238462643383279502884L;
    std::vector<long double> T((size_t)n * n);
    for (int q = 0; q < n; ++q)
        for (int e = 0; e < n; ++e) {
            long double v;
            const long double x = e + 0.5L;
            switch (kind) {
            case K_P:
                if (q == 0) v = 1;
                else if (q == 1) v = (e & 1) ? -1 : 1;
                else if (q % 2 == 0) v = cosl(2 * pi * (q / 2) * e / n);
                else v = -sinl(2 * pi * (q / 2) * e / n);
                break;
            case K_NN: v = cosl(pi * q * x / n); break;
            case K_DD: v = sinl(pi * (q + 1) * x / n); break;
            case K_ND: v = cosl(pi * (2 * q + 1) * (2 * e + 1) / (4.0L * n)); break;
            default: v = sinl(pi * (2 * q + 1) * (2 * e + 1) / (4.0L * n)); break;
            }
            T[(size_t)q * n + e] = v;
        }
    return T;
}

// The inverse B = s T^{-1} = s T^T diag(1/|row_q|^2), as rows B[e][q].
inline std::vector<long double> dense_inverse(int kind, int n)
{
    std::vector<long double> T = dense_forward(kind, n), B((size_t)n * n);
    const long double s = xform_scale(kind, n);
    for (int q = 0; q < n; ++q) {
        long double nn = 0;
        for (int e = 0; e < n; ++e) nn += T[(size_t)q * n + e] * T[(size_t)q * n + e];
        for (int e = 0; e < n; ++e) B[(size_t)e * n + q] = s * T[(size_t)q * n + e] / nn;
    }
    return B;
}

// dense transforms apply to the cell-centred kinds, n = 128 .. 512 in steps of 128
inline bool dense_ok(int kind, int n) { return kind <= K_DN && n >= 128 && n <= 512 && n % 128 == 0; }

}  // namespace cans

// zsolve_core.h -- the z direction of the solver: one tridiagonal system per
// spectral column (eq. (poi_reduced), Section 2), solved in FP64 by Gauss
// elimination without pivoting (Thomas), and the FP64 residual of eq. (poi)
// used by iterative refinement.  Host/device functions so the serial host
// build runs the same arithmetic in the tests.
#pragma once

#include "xform_core.h"

namespace cans {

// Column systems, row k:  a_k p_{k-1} + (b_k + lam) p_k + c_k p_{k+1} = s f_k
//   lam = lamx[i] + lamy[j] (mu/h^2 of the x and y transforms), s = scale.
// a/b/c carry the z boundary folding (wall rows: outer coefficient 0; periodic:
// corner couplings a_0 -> p_{nz-1}, c_{nz-1} -> p_0).
struct ZArgs {
    int nx, ny, nz;
    const double *za, *zb, *zc;
    const double *lamx, *lamy;
    const double *dzf;
    double wsum;        // sum of dzf
    double scale;       // 1/(s_x s_y), the transforms' normalisation
    int cyclic;         // periodic z (nz >= 3)
    int singular;       // every axis P or NN: column (0,0) is singular
    double *wc;         // workspace: elimination multipliers c'_k (FP64 field)
    double *wd;         // workspace: modified right-hand side d'_k (FP64 field)
    double *wz;         // workspace: second right-hand side (cyclic only)
    double *removed;    // singular: receives the removed weighted mean (or null)
};

template <typename T> CANS_HD double ld(const T *p, size_t i) { return (double)p[i]; }
template <typename T> CANS_HD void st(T *p, size_t i, double v) { p[i] = (T)v; }

// The singular column (kx = ky = 0 with z periodic or Neumann-Neumann):
// project the rhs by its dzf-weighted mean (dzf is the left null vector of the
// z operator), solve with the last equation replaced by p_{nz-1} = 0 (the
// periodic corner then multiplies the pinned unknown), and shift the result
// to zero weighted mean.
// wc, wd: workspace of the column, level k at wc[k * ws], wd[k * ws]
template <typename T>
CANS_HD void zsolve_singular_ws(size_t col, T *data, const ZArgs &a, double *wc, double *wd, size_t ws)
{
    const size_t plane = (size_t)a.nx * a.ny;
    const int nz = a.nz;
    double s = 0;
    for (int k = 0; k < nz; ++k) s += a.dzf[k] * (a.scale * ld(data, col + plane * k));
    const double m = s / a.wsum;
    if (a.removed) *a.removed = m;
    if (nz == 1) {
        st(data, col, 0.0);
        return;
    }
    double piv = a.zb[0];
    double d = (a.scale * ld(data, col) - m) / piv;
    wd[0] = d;
    for (int k = 1; k < nz; ++k) {
        const double w = a.zc[k - 1] / piv;
        wc[k * ws] = w;
        const bool last = (k == nz - 1);
        const double ak = last ? 0.0 : a.za[k];
        piv = (last ? 1.0 : a.zb[k]) - ak * w;
        const double rhs = last ? 0.0 : a.scale * ld(data, col + plane * k) - m;
        d = (rhs - ak * d) / piv;
        wd[k * ws] = d;
    }
    double x = d, s2 = a.dzf[nz - 1] * x;
    for (int k = nz - 2; k >= 0; --k) {
        x = wd[k * ws] - wc[(k + 1) * ws] * x;
        wd[k * ws] = x;
        s2 += a.dzf[k] * x;
    }
    wd[(nz - 1) * ws] = d;
    const double m2 = s2 / a.wsum;
    for (int k = 0; k < nz; ++k) st(data, col + plane * k, wd[k * ws] - m2);
}

// One spectral column, in place in `data` (T = double or float storage).
template <typename T>
CANS_HD void zsolve_singular(size_t col, T *data, const ZArgs &a)
{
    const size_t plane = (size_t)a.nx * a.ny;
    zsolve_singular_ws(col, data, a, a.wc + col, a.wd + col, plane);
}

template <typename T>
CANS_HD void zsolve_column(size_t col, T *data, const ZArgs &a)
{
    const size_t plane = (size_t)a.nx * a.ny;
    const int nz = a.nz;
    const int i = (int)(col % a.nx), j = (int)(col / a.nx);
    if (a.singular && i == 0 && j == 0) {
        zsolve_singular(col, data, a);
        return;
    }
    const double lam = a.lamx[i] + a.lamy[j];
    if (!a.cyclic) {
        double piv = a.zb[0] + lam;
        double d = a.scale * ld(data, col) / piv;
        a.wd[col] = d;
        for (int k = 1; k < nz; ++k) {
            const size_t e = col + plane * k;
            const double w = a.zc[k - 1] / piv;
            a.wc[e] = w;
            piv = a.zb[k] + lam - a.za[k] * w;
            d = (a.scale * ld(data, e) - a.za[k] * d) / piv;
            a.wd[e] = d;
        }
        double x = d;
        st(data, col + plane * (nz - 1), x);
        for (int k = nz - 2; k >= 0; --k) {
            const size_t e = col + plane * k;
            x = a.wd[e] - a.wc[e + plane] * x;
            st(data, e, x);
        }
        return;
    }
    // periodic z, Sherman-Morrison: A = A' + u v^T, u = (g, 0.., c_{n-1}),
    // v = (1, 0.., a_0/g), g = -(b_0 + lam); x = y - z (v.y)/(1 + v.z) with
    // A' y = f and A' z = u sharing one elimination.
    const double g = -(a.zb[0] + lam);
    const double cn = a.zc[nz - 1], a0 = a.za[0];
    double piv = a.zb[0] + lam - g;
    double dy = a.scale * ld(data, col) / piv, dz = g / piv;
    a.wd[col] = dy;
    a.wz[col] = dz;
    for (int k = 1; k < nz; ++k) {
        const size_t e = col + plane * k;
        const double w = a.zc[k - 1] / piv;
        a.wc[e] = w;
        const double bk = (k == nz - 1) ? a.zb[k] + lam - cn * a0 / g : a.zb[k] + lam;
        piv = bk - a.za[k] * w;
        dy = (a.scale * ld(data, e) - a.za[k] * dy) / piv;
        dz = ((k == nz - 1 ? cn : 0.0) - a.za[k] * dz) / piv;
        a.wd[e] = dy;
        a.wz[e] = dz;
    }
    const double yl = dy, zl = dz;
    double y = dy, z = dz;
    for (int k = nz - 2; k >= 0; --k) {
        const size_t e = col + plane * k;
        y = a.wd[e] - a.wc[e + plane] * y;
        z = a.wz[e] - a.wc[e + plane] * z;
        a.wd[e] = y;
        a.wz[e] = z;
    }
    const double fac = (y + a0 / g * yl) / (1.0 + z + a0 / g * zl);
    for (int k = 0; k < nz; ++k) {
        const size_t e = col + plane * k;
        st(data, e, a.wd[e] - fac * a.wz[e]);
    }
}

// ---------------------------------------------------------------------------
// FP64 residual r = (f - mf) - L_h p at one point, eq. (poi) with the z part
// in conservative form; neighbours across a face follow its ghost rule.
struct LapArgs {
    int nx, ny, nz;
    int bc[6];
    double idx2, idy2;
    const double *zaf;  // 1/(dzc_{k-1} dzf_k), unfolded (ghost spacing at walls)
    const double *zcf;  // 1/(dzc_k dzf_k), unfolded
    double shift;       // Helmholtz shift s: the operator is L_h + s
};

// z neighbour across a wall by its ghost rule: periodic wraps, Neumann
// mirrors, Dirichlet is antisymmetric.  A face-located z field (code 3)
// takes the antisymmetric ghost too, with its wall coupling halved in the
// tables: (a/2)(w - (-w)) = a (w - 0) exactly, its zero wall value.
CANS_HD double ghost(int bc, double inner, double wrap)
{
    return bc == 0 ? wrap : (bc == 1 ? inner : -inner);
}

// x and y: index and sign of the value that stands beyond the lower (lo) or
// upper end of a line of n values.  Periodic wraps, Neumann mirrors,
// Dirichlet mirrors with the sign flipped; a field on the faces of the axis
// is zero beyond a Dirichlet face (sign 0) and mirrored about a Neumann face
// it sits on (the second value from that end).
CANS_HD void beyond(int bc, bool lo, int n, int &idx, double &sg)
{
    sg = 1.0;
    switch (bc) {
    case 0: idx = lo ? n - 1 : 0; break;
    case 1: idx = lo ? 0 : n - 1; break;
    case 2: idx = lo ? 0 : n - 1; sg = -1.0; break;
    case 3: idx = lo ? 0 : n - 1; sg = 0.0; break;
    default: idx = lo ? 1 : n - 2; break;
    }
}

// the value beyond an end of the line through element e (index i, stride st)
CANS_HD double across(int bc, bool lo, const double *p, size_t e, int i, int n, size_t st)
{
    int gi;
    double sg;
    beyond(bc, lo, n, gi, sg);
    return sg * p[(ptrdiff_t)e + ((ptrdiff_t)gi - i) * (ptrdiff_t)st];
}

CANS_HD double lap_point(const double *p, int i, int j, int k, const LapArgs &a)
{
    const size_t sx = 1, sy = (size_t)a.nx, sz = (size_t)a.nx * a.ny;
    const size_t e = i + sy * j + sz * k;
    if (i > 0 && i < a.nx - 1 && j > 0 && j < a.ny - 1 && k > 0 && k < a.nz - 1) {
        // interior: no ghost cells
        const double *q = p + e;
        const double c = q[0];
        return (q[-1] - 2.0 * c + q[1]) * a.idx2 + (q[-(long)sy] - 2.0 * c + q[sy]) * a.idy2
             + a.zcf[k] * (q[sz] - c) - a.zaf[k] * (c - q[-(long)sz]) + a.shift * c;
    }
    const double c = p[e];
    const double xm = i > 0 ? p[e - sx] : across(a.bc[0], true, p, e, i, a.nx, sx);
    const double xp = i < a.nx - 1 ? p[e + sx] : across(a.bc[1], false, p, e, i, a.nx, sx);
    const double ym = j > 0 ? p[e - sy] : across(a.bc[2], true, p, e, j, a.ny, sy);
    const double yp = j < a.ny - 1 ? p[e + sy] : across(a.bc[3], false, p, e, j, a.ny, sy);
    const double zm = k > 0 ? p[e - sz] : ghost(a.bc[4], c, p[e + (a.nz - 1) * sz]);
    const double zp = k < a.nz - 1 ? p[e + sz] : ghost(a.bc[5], c, p[e - (a.nz - 1) * sz]);
    return (xm - 2.0 * c + xp) * a.idx2 + (ym - 2.0 * c + yp) * a.idy2
         + a.zcf[k] * (zp - c) - a.zaf[k] * (c - zm) + a.shift * c;
}

}  // namespace cans

namespace cans {

// ---------------------------------------------------------------------------
// Partitioned column solve (no workspace).  A block owns 64 adjacent columns
// (lane = column) and splits z into S segments (wave = segment), each of
// m <= MMAX levels held in registers.  Within a segment, with the outside
// neighbours xL = x_{k0-1} and xR = x_{k1}:
//   top-down elimination   ->  x_{k1-1} + C xL + E xR = F
//   bottom-up elimination  ->  x_{k0}   + A xL + B xR = D
// The 2S end unknowns (u_s = x_{k0}, v_s = x_{k1-1}) satisfy
//   u_s + A_s v_{s-1} + B_s u_{s+1} = D_s,   v_s + C_s v_{s-1} + E_s u_{s+1} = F_s,
// a block-tridiagonal system with 2x2 blocks whose coupling matrices have one
// non-zero column each; it is eliminated in one pass over the segments and
// back-substituted.  Each segment then re-runs its top-down sweep with xL
// known (reusing the stored reciprocal pivots) and back-substitutes from xR.
// Gauss elimination without pivoting throughout (diagonally dominant), FP64.
// The singular column of a singular problem is not part of it: the kernel
// solves that column apart (zsolve_singular_ws).

// 1/x as v_rcp_f64 refined by two Newton steps on the device.
CANS_HD double rcp64(double x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
#else
    return 1.0 / x;
#endif
}

// Materialise x here (device only).  The fill-in recurrences below are pure
// running products; left alone, the compiler defers them to the end of the
// unrolled sweep, which keeps every level's pivot and coefficient live at once
// and runs the block out of registers.
CANS_HD void zp_pin(double &x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    asm volatile("" : "+v"(x));
#else
    (void)x;
#endif
}

struct ZSeg {
    int k0, m;
};

CANS_HD ZSeg zseg(int nz, int S, int w)
{
    const int base = nz / S, rem = nz % S;
    ZSeg s;
    s.k0 = w * base + (w < rem ? w : rem);
    s.m = base + (w < rem ? 1 : 0);
    return s;
}

// Row coefficients of level k for a lane.  CYC (periodic z): the rows of the
// tridiagonal part A' of the cyclic matrix A = A' + u v^T (Sherman-Morrison,
// u = (gam, 0.., c_{n-1}), v = (1, 0.., a_0/gam), gam = -(b_0 + lam)): the
// wrap couplings dropped and folded into the first and last diagonals.
template <bool CYC>
CANS_HD void zrow(const ZArgs &a, int k, double lam, double gam, double &ak, double &bk, double &ck)
{
    ak = a.za[k];
    bk = a.zb[k] + lam;
    ck = a.zc[k];
    if (CYC) {
        if (k == 0) { ak = 0.0; bk -= gam; }
        if (k == a.nz - 1) { ck = 0.0; bk -= a.zc[k] * a.za[0] / gam; }
    }
}

// Level k of a column padded to whole segments (non-periodic z): beyond nz
// the rows (0, -1, 0) with a zero rhs.  The last real row has c = 0, so the
// padding decouples exactly, solves to zero (its pivot -1 + lam has modulus
// >= 1 as lam <= 0) and leaves the real levels as they are.
CANS_HD void zpad_row(const ZArgs &a, int k, double &ak, double &bk, double &ck)
{
    const bool real = k < a.nz;
    ak = real ? a.za[k] : 0.0;
    bk = real ? a.zb[k] : -1.0;
    ck = real ? a.zc[k] : 0.0;
}

// FULL: every segment has exactly MMAX levels, so the level guards fold away.
// PAD (with FULL, non-periodic): the segments cover S*MMAX >= nz levels, the
// tables hold the padding rows of zpad_row, and only the loads and stores
// test k < nz.
// CYC: a second right-hand side u (Sherman-Morrison) is carried beside f.
template <int MMAX, bool CYC = false>
struct ZLane {
    double f[MMAX];                // rhs, later the forward-swept rhs, later x
    double r[MMAX];                // reciprocal pivots of the top-down sweep
    double u[CYC ? MMAX : 1];      // CYC: u, later A'^{-1} u
    double lam, gam;
    bool valid;
};

// load the segment's rhs (scaled) and the column's lambda
template <int MMAX, bool FULL, bool PAD = false, typename T, bool CYC>
CANS_HD void zp_load(ZLane<MMAX, CYC> &L, const T *data, const ZArgs &a, size_t col, ZSeg sg)
{
    static_assert(!PAD || (FULL && !CYC), "padding is for full non-periodic segments");
    const size_t plane = (size_t)a.nx * a.ny;
    // the singular column (singular problems, column 0) is solved apart
    L.valid = col < plane && !(a.singular && col == 0);
    // 32-bit index arithmetic: a plane holds at most 4096 x 4096 columns
    const unsigned cu = L.valid ? (unsigned)col : 0u, nxu = (unsigned)a.nx;
    L.lam = L.valid ? a.lamx[cu % nxu] + a.lamy[cu / nxu] : -1.0;
    L.gam = -(a.zb[0] + L.lam);
    const T *ptr = data + (L.valid ? col : 0) + plane * sg.k0;
#pragma unroll
    for (int t = 0; t < MMAX; ++t) {
        if (FULL || t < sg.m) {
            L.f[t] = L.valid && (!PAD || sg.k0 + t < a.nz) ? a.scale * (double)ptr[0] : 0.0;
            if constexpr (CYC) {
                const int k = sg.k0 + t;
                L.u[t] = (k == 0 ? L.gam : 0.0) + (k == a.nz - 1 ? a.zc[a.nz - 1] : 0.0);
            }
        }
        ptr += plane;
    }
}

// step 1: both sweeps over the segment; out[0..5] = A, B, C, D, E, F, and
// for CYC out[6], out[7] = D, F of the second right-hand side.
// The top-down sweep (level i) and the bottom-up sweep (level MMAX-1-i, live
// once it is below m) run in one unrolled loop: two independent dependency
// chains for the scheduler to interleave.
template <int MMAX, bool FULL, bool CYC>
CANS_HD void zp_reduce(ZLane<MMAX, CYC> &L, const ZArgs &a, ZSeg sg, double *out)
{
    double cp = 0, d = 0, g = 0, d2 = 0;    // top-down: c', d' (f, u), fill-in of xL
    double ep = 0, dd = 0, h = 0, dd2 = 0;  // bottom-up: a'', d'' (f, u), fill-in of xR
#pragma unroll
    for (int i = 0; i < MMAX; ++i) {
        const int t = i;
        if (FULL || t < sg.m) {
            double ak, bk, ck;
            zrow<CYC>(a, sg.k0 + t, L.lam, L.gam, ak, bk, ck);
            const double rr = rcp64(t == 0 ? bk : bk - ak * cp);
            L.r[t] = rr;
            d = (t == 0 ? L.f[t] : L.f[t] - ak * d) * rr;
            if constexpr (CYC) {
                d2 = (t == 0 ? L.u[t] : L.u[t] - ak * d2) * rr;
                zp_pin(d2);  // u is zero inside: a running product
            }
            g = (t == 0 ? ak : -ak * g) * rr;
            zp_pin(g);
            cp = ck * rr;
        }
        const int u = MMAX - 1 - i;
        if (FULL || u < sg.m) {
            double ak, bk, ck;
            zrow<CYC>(a, sg.k0 + u, L.lam, L.gam, ak, bk, ck);
            const bool last = FULL ? (u == MMAX - 1) : (u == sg.m - 1);
            const double rr = rcp64(last ? bk : bk - ck * ep);
            dd = (last ? L.f[u] : L.f[u] - ck * dd) * rr;
            if constexpr (CYC) {
                dd2 = (last ? L.u[u] : L.u[u] - ck * dd2) * rr;
                zp_pin(dd2);
            }
            h = (last ? ck : -ck * h) * rr;
            zp_pin(h);
            ep = ak * rr;
        }
    }
    out[0] = ep;  // A
    out[1] = h;   // B
    out[2] = g;   // C
    out[3] = dd;  // D
    out[4] = cp;  // E
    out[5] = d;   // F
    if constexpr (CYC) {
        out[6] = dd2;
        out[7] = d2;
    }
}

// step 2: the reduced system of one column over its S segments.
// c(s, q) addresses coefficient q of segment s; u(s), v(s) receive the ends
// (CYC: u2(s), v2(s) those of the second right-hand side, whose D, F are
// c(s, 6), c(s, 7)).
template <bool CYC, typename Coef, typename OutU, typename OutV, typename OutU2, typename OutV2>
CANS_HD void zp_interface(int S, Coef c, OutU uo, OutV vo, OutU2 uo2, OutV2 vo2)
{
    // forward: v_s = y2 - g2 u_{s+1}; the next segment's coefficients are
    // read one step ahead so their latency overlaps the recurrence
    double g2p = 0, y2p = 0, w2p = 0;
    double A = c(0, 0), B = c(0, 1), C = c(0, 2), D = c(0, 3), E = c(0, 4), F = c(0, 5);
    double D2 = CYC ? c(0, 6) : 0.0, F2 = CYC ? c(0, 7) : 0.0;
    for (int s = 0; s < S; ++s) {
        const int sn = s + 1 < S ? s + 1 : s;
        const double An = c(sn, 0), Bn = c(sn, 1), Cn = c(sn, 2), Dn = c(sn, 3), En = c(sn, 4), Fn = c(sn, 5);
        const double D2n = CYC ? c(sn, 6) : 0.0, F2n = CYC ? c(sn, 7) : 0.0;
        const double inv = rcp64(1.0 - A * g2p);
        const double y1 = (D - A * y2p) * inv;
        const double y2 = (F - C * y2p) + C * g2p * y1;
        const double g1 = B * inv;
        const double g2 = E + C * g2p * g1;
        c(s, 0) = y1; c(s, 1) = y2; c(s, 2) = g1; c(s, 3) = g2;
        if constexpr (CYC) {
            const double w1 = (D2 - A * w2p) * inv;
            const double w2 = (F2 - C * w2p) + C * g2p * w1;
            c(s, 6) = w1; c(s, 7) = w2;
            w2p = w2;
        }
        g2p = g2;
        y2p = y2;
        A = An; B = Bn; C = Cn; D = Dn; E = En; F = Fn; D2 = D2n; F2 = F2n;
    }
    // backward: u_s = y1 - g1 u_{s+1}, v_s = y2 - g2 u_{s+1}
    double un = 0, un2 = 0;
    double y1 = c(S - 1, 0), y2 = c(S - 1, 1), g1 = c(S - 1, 2), g2 = c(S - 1, 3);
    double w1 = CYC ? c(S - 1, 6) : 0.0, w2 = CYC ? c(S - 1, 7) : 0.0;
    for (int s = S - 1; s >= 0; --s) {
        const int sp = s > 0 ? s - 1 : 0;
        const double y1n = c(sp, 0), y2n = c(sp, 1), g1n = c(sp, 2), g2n = c(sp, 3);
        const double w1n = CYC ? c(sp, 6) : 0.0, w2n = CYC ? c(sp, 7) : 0.0;
        const double u = y1 - g1 * un;
        uo(s) = u;
        vo(s) = y2 - g2 * un;
        un = u;
        if constexpr (CYC) {
            const double u2 = w1 - g1 * un2;
            uo2(s) = u2;
            vo2(s) = w2 - g2 * un2;
            un2 = u2;
        }
        y1 = y1n; y2 = y2n; g1 = g1n; g2 = g2n; w1 = w1n; w2 = w2n;
    }
}

// step 3: x of the segment from its outside neighbours xL, xR (CYC: also the
// second right-hand side's, xL2, xR2)
template <int MMAX, bool FULL, bool CYC>
CANS_HD void zp_finish(ZLane<MMAX, CYC> &L, const ZArgs &a, ZSeg sg, double xL, double xR, double xL2 = 0.0,
                       double xR2 = 0.0)
{
    double d = xL, d2 = xL2;
#pragma unroll
    for (int t = 0; t < MMAX; ++t) {
        if (FULL || t < sg.m) {
            double ak, bk, ck;
            zrow<CYC>(a, sg.k0 + t, L.lam, L.gam, ak, bk, ck);
            d = (L.f[t] - ak * d) * L.r[t];
            L.f[t] = d;
            if constexpr (CYC) {
                d2 = (L.u[t] - ak * d2) * L.r[t];
                zp_pin(d2);
                L.u[t] = d2;
            }
        }
    }
    double x = xR, x2 = xR2;
#pragma unroll
    for (int t = MMAX - 1; t >= 0; --t) {
        if (FULL || t < sg.m) {
            double ak, bk, ck;
            zrow<CYC>(a, sg.k0 + t, L.lam, L.gam, ak, bk, ck);
            x = L.f[t] - ck * L.r[t] * x;
            L.f[t] = x;
            if constexpr (CYC) {
                x2 = L.u[t] - ck * L.r[t] * x2;
                zp_pin(x2);
                L.u[t] = x2;
            }
        }
    }
}

// CYC: first and last values of y = A'^{-1} f and z = A'^{-1} u in this
// segment (meaningful in the first and the last segment)
template <int MMAX, bool FULL, bool CYC>
CANS_HD void zp_ends(const ZLane<MMAX, CYC> &L, ZSeg sg, double *y0, double *z0, double *yl, double *zl)
{
    *y0 = L.f[0];
    *z0 = CYC ? L.u[0] : 0.0;
    *yl = 0.0;
    *zl = 0.0;
#pragma unroll
    for (int t = 0; t < MMAX; ++t)
        if ((FULL && t == MMAX - 1) || (!FULL && t == sg.m - 1)) {
            *yl = L.f[t];
            if constexpr (CYC) *zl = L.u[t];
        }
}

// CYC: x = y - z (v.y) / (1 + v.z) with v = (1, 0.., a_0/gam)
template <int MMAX, bool FULL, bool CYC>
CANS_HD void zp_sherman_morrison(ZLane<MMAX, CYC> &L, const ZArgs &a, ZSeg sg, double y0, double z0, double yl,
                                 double zl)
{
    if constexpr (CYC) {
        const double w = a.za[0] / L.gam;
        const double fac = (y0 + w * yl) / (1.0 + z0 + w * zl);
#pragma unroll
        for (int t = 0; t < MMAX; ++t)
            if (FULL || t < sg.m) L.f[t] -= fac * L.u[t];
    }
}

template <int MMAX, bool FULL, bool PAD = false, typename T, bool CYC>
CANS_HD void zp_store(const ZLane<MMAX, CYC> &L, T *data, const ZArgs &a, size_t col, ZSeg sg)
{
    if (!L.valid) return;
    const size_t plane = (size_t)a.nx * a.ny;
    T *ptr = data + col + plane * sg.k0;
#pragma unroll
    for (int t = 0; t < MMAX; ++t) {
        if ((FULL || t < sg.m) && (!PAD || sg.k0 + t < a.nz)) ptr[0] = (T)L.f[t];
        ptr += plane;
    }
}

// ---------------------------------------------------------------------------
// Single-sweep form of the segment reduction (non-periodic z).  The top-down
// elimination of a segment with its outside neighbours xL, xR kept symbolic,
//   x_t = d_t - g_t xL - cp_t x_{t+1},
// also gives the first row by back-substituting symbolically:
//   x_0 = sum_t P_t (d_t - g_t xL) + P_m xR,   P_t = prod_{j<t} (-cp_j),
// so one sweep yields all six coefficients of the interface relations
//   x_{k0} + A xL + B xR = D,   x_{k1-1} + C xL + E xR = F
// with A = sum P_t g_t, B = -P_m, D = sum P_t d_t, C = g_{m-1}, E = cp_{m-1},
// F = d_{m-1}.  Only the reciprocal pivots r_t are kept for the finish.  For
// the operators here b + lam < 0 < a, c, so every P_t and every g_t has one
// sign: the sums for A and B do not cancel.
// fv(t): scaled rhs of level t; za/zb/zc: the segment's first level.
template <int MMAX, typename FV>
CANS_HD void zp_sweep_reduce(const FV &fv, const double *za, const double *zb, const double *zc, double lam,
                             double (&r)[MMAX], double (&out)[6])
{
    double cp = 0, d = 0, g = 0, P = 1, Ds = 0, As = 0;
    // the next level's coefficients are read one level ahead
    double an = za[0], bn = zb[0], cn = zc[0];
    for (int t = 0; t < MMAX; ++t) {
        const double ak = an, bk = bn + lam, ck = cn;
        if (t + 1 < MMAX) {
            an = za[t + 1];
            bn = zb[t + 1];
            cn = zc[t + 1];
        }
        const double rr = rcp64(t == 0 ? bk : bk - ak * cp);
        r[t] = rr;
        d = (t == 0 ? fv(t) : fv(t) - ak * d) * rr;
        g = (t == 0 ? ak : -ak * g) * rr;
        zp_pin(g);
        Ds = fma(P, d, Ds);
        As = fma(P, g, As);
        cp = ck * rr;
        P = -P * cp;
        zp_pin(P);
    }
    out[0] = As;
    out[1] = -P;
    out[2] = g;
    out[3] = Ds;
    out[4] = cp;
    out[5] = d;
}

// x of the segment from its outside neighbours: the top-down sweep again with
// xL known (stored reciprocal pivots), then back-substitution from xR.
template <int MMAX, typename FV>
CANS_HD void zp_sweep_finish(const FV &fv, const double *za, const double *zc, const double (&r)[MMAX], double xL,
                             double xR, double (&x)[MMAX])
{
    double d = xL;
    double an = za[0];
    for (int t = 0; t < MMAX; ++t) {
        const double ak = an;
        if (t + 1 < MMAX) an = za[t + 1];
        d = (fv(t) - ak * d) * r[t];
        x[t] = d;
    }
    double xx = xR;
    double cn = zc[MMAX - 1];
    for (int t = MMAX - 1; t >= 0; --t) {
        const double ck = cn;
        if (t > 0) cn = zc[t - 1];
        xx = x[t] - ck * r[t] * xx;
        x[t] = xx;
    }
}

// The interface system of one column solved from both ends at once.  The top
// role eliminates over segments 0 .. S/2-1 exactly as zp_interface does
// (v_s = y2 - g2 u_{s+1}, u_s = y1 - g1 u_{s+1}); the bottom role eliminates
// upwards over S-1 .. S/2 (u_s = p1 - h1 v_{s-1}, v_s = p2 - h2 v_{s-1}).  The
// bottom recurrence is the top one with the coefficients (A,B,C,D,E,F) read as
// (E,C,B,F,A,D) and the results (y1,y2,g1,g2) standing for (p2,p1,h2,h1), so
// one code path serves both.  The two chains meet between segments S/2-1 and
// S/2 (v_{S/2-1} = y2 - g2 u_{S/2}, u_{S/2} = p1 - h1 v_{S/2-1}), then each role
// substitutes back over its half.  Coefficients are read NB steps at a time.
// C(q, s): coefficient q of segment s of this column; results u_s -> C(4, s),
// v_s -> C(5, s).
CANS_HD int zp_ends_steps(int S, bool bot) { return bot ? S - S / 2 : S / 2; }

template <int NB, typename Cf>
CANS_HD void zp_ends_forward(int S, bool bot, Cf C, double &y2p, double &g2p)
{
    const int n = zp_ends_steps(S, bot), nmax = S - S / 2;
    const int qA = bot ? 4 : 0, qB = bot ? 2 : 1, qC = bot ? 1 : 2, qD = bot ? 5 : 3, qE = bot ? 0 : 4, qF = bot ? 3 : 5;
    y2p = 0;
    g2p = 0;
#pragma unroll 1
    for (int b0 = 0; b0 < nmax; b0 += NB) {
        double A[NB], B[NB], Cc[NB], D[NB], E[NB], F[NB];
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            const int i = b0 + j < n ? b0 + j : n - 1;
            const int s = bot ? S - 1 - i : i;
            A[j] = C(qA, s); B[j] = C(qB, s); Cc[j] = C(qC, s);
            D[j] = C(qD, s); E[j] = C(qE, s); F[j] = C(qF, s);
        }
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            const int i = b0 + j;
            if (i < n) {
                const int s = bot ? S - 1 - i : i;
                const double inv = rcp64(1.0 - A[j] * g2p);
                const double y1 = (D[j] - A[j] * y2p) * inv;
                const double cg = Cc[j] * g2p;
                const double y2 = (F[j] - Cc[j] * y2p) + cg * y1;
                const double g1 = B[j] * inv;
                const double g2 = E[j] + cg * g1;
                C(0, s) = y1;
                C(1, s) = y2;
                C(2, s) = g1;
                C(3, s) = g2;
                g2p = g2;
                y2p = y2;
            }
        }
    }
}

// the unknown next to the meeting point on this role's side of the other
// role's last relation: top gets u_{S/2}, bottom gets v_{S/2-1}
CANS_HD double zp_ends_meet(double y2, double g2, double y2o, double g2o)
{
    return (y2o - g2o * y2) * rcp64(1.0 - g2 * g2o);
}

template <int NB, typename Cf>
CANS_HD void zp_ends_backward(int S, bool bot, Cf C, double prev)
{
    const int n = zp_ends_steps(S, bot), nmax = S - S / 2;
    const int q1 = bot ? 5 : 4, q2 = bot ? 4 : 5;
#pragma unroll 1
    for (int b0 = 0; b0 < nmax; b0 += NB) {
        double Y1[NB], Y2[NB], G1[NB], G2[NB];
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            const int i0 = n - 1 - (b0 + j);
            const int i = i0 >= 0 ? i0 : 0;
            const int s = bot ? S - 1 - i : i;
            Y1[j] = C(0, s); Y2[j] = C(1, s); G1[j] = C(2, s); G2[j] = C(3, s);
        }
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            const int i0 = n - 1 - (b0 + j);
            if (i0 >= 0) {
                const int s = bot ? S - 1 - i0 : i0;
                const double o1 = Y1[j] - G1[j] * prev;
                const double o2 = Y2[j] - G2[j] * prev;
                C(q1, s) = o1;
                C(q2, s) = o2;
                prev = o1;
            }
        }
    }
}

// Shape of the partitioned solve for nz: register depth per lane, columns
// per block and threads per block (segments = threads/64 * 64/cpb).
//   nz <= 128: 64 columns, segments of <= 8 levels;
//   nz <= 256: 64 columns, segments of <= 16 levels;
//   nz <= 512: 32 columns (two segments per wave), segments of <= 16 levels.
// mmax = 0 when nz > 512 (the plain elimination with a workspace is used
// then).  Periodic z uses the same shapes with the cyclic (CYC) form.
struct ZPart {
    int mmax, cpb, threads;
};

inline ZPart zpart_shape(int nz)
{
    if (nz <= 128) return ZPart{8, 64, 64 * ((nz + 7) / 8)};
    if (nz <= 256) return ZPart{16, 64, 64 * ((nz + 15) / 16)};
    if (nz <= 512) {
        const int segs = (nz + 15) / 16;          // <= 32, two per wave
        return ZPart{16, 32, 64 * ((segs + 1) / 2)};
    }
    return ZPart{0, 0, 0};
}

// Periodic z carries a second right-hand side (Sherman-Morrison): segments of
// <= 8 levels, 64 columns, up to nz = 128.  Deeper periodic columns use the
// plain elimination: there the combination of the two partitioned solutions
// lost up to 3x the accuracy of the sequential one on the ill-conditioned
// low-wavenumber columns (measured against the long-double oracle).
inline ZPart zpart_shape_cyc(int nz)
{
    if (nz <= 128) return ZPart{8, 64, 64 * ((nz + 7) / 8)};
    return ZPart{0, 0, 0};
}

inline ZPart zpart_shape(int nz, bool cyclic) { return cyclic ? zpart_shape_cyc(nz) : zpart_shape(nz); }

inline int zpart_mmax(int nz) { return zpart_shape(nz).mmax; }

}  // namespace cans

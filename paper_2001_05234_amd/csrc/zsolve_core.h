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
template <typename T>
CANS_HD void zsolve_singular(size_t col, T *data, const ZArgs &a)
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
    a.wd[col] = d;
    for (int k = 1; k < nz; ++k) {
        const double w = a.zc[k - 1] / piv;
        a.wc[col + plane * k] = w;
        const bool last = (k == nz - 1);
        const double ak = last ? 0.0 : a.za[k];
        piv = (last ? 1.0 : a.zb[k]) - ak * w;
        const double rhs = last ? 0.0 : a.scale * ld(data, col + plane * k) - m;
        d = (rhs - ak * d) / piv;
        a.wd[col + plane * k] = d;
    }
    double x = d, s2 = a.dzf[nz - 1] * x;
    for (int k = nz - 2; k >= 0; --k) {
        x = a.wd[col + plane * k] - a.wc[col + plane * (k + 1)] * x;
        a.wd[col + plane * k] = x;
        s2 += a.dzf[k] * x;
    }
    a.wd[col + plane * (nz - 1)] = d;
    const double m2 = s2 / a.wsum;
    for (int k = 0; k < nz; ++k) st(data, col + plane * k, a.wd[col + plane * k] - m2);
}

// One spectral column, in place in `data` (T = double or float storage).
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
};

CANS_HD double ghost(int bc, double inner, double wrap)
{
    return bc == 0 ? wrap : (bc == 1 ? inner : -inner);
}

CANS_HD double lap_point(const double *p, int i, int j, int k, const LapArgs &a)
{
    const size_t sx = 1, sy = (size_t)a.nx, sz = (size_t)a.nx * a.ny;
    const size_t e = i + sy * j + sz * k;
    const double c = p[e];
    const double xm = i > 0 ? p[e - sx] : ghost(a.bc[0], c, p[e + (a.nx - 1) * sx]);
    const double xp = i < a.nx - 1 ? p[e + sx] : ghost(a.bc[1], c, p[e - (a.nx - 1) * sx]);
    const double ym = j > 0 ? p[e - sy] : ghost(a.bc[2], c, p[e + (a.ny - 1) * sy]);
    const double yp = j < a.ny - 1 ? p[e + sy] : ghost(a.bc[3], c, p[e - (a.ny - 1) * sy]);
    const double zm = k > 0 ? p[e - sz] : ghost(a.bc[4], c, p[e + (a.nz - 1) * sz]);
    const double zp = k < a.nz - 1 ? p[e + sz] : ghost(a.bc[5], c, p[e - (a.nz - 1) * sz]);
    return (xm - 2.0 * c + xp) * a.idx2 + (ym - 2.0 * c + yp) * a.idy2
         + a.zcf[k] * (zp - c) - a.zaf[k] * (c - zm);
}

}  // namespace cans

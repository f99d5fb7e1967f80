// cans_emu.cpp -- host build of the GPU library's kernel arithmetic, for the
// CPU test suite.  It runs the same tile transforms (xform_core.h), the same
// column solve and residual (zsolve_core.h) and the same tables (tables.h)
// serially on the host, tile by tile with the kernels' tile shapes, so the
// index math of the HIP path is checked against the oracle without a GPU.
// Test infrastructure: nothing in the library uses it.
#include <cmath>
#include <cstring>
#include <vector>

#include "tables.h"
#include "zsolve_core.h"

using namespace cans;

namespace {

struct NoSync {
    void operator()() const {}
};

// transform along x (axis 0) or y (axis 1) of a (nz, ny, nx) field, in place,
// tile by tile with the kernels' tile shapes (two tiles: out of place)
template <int KIND, bool FWD, int AXIS, typename T>
void xform_k(const XGeom &g, int nx, int ny, int nz, std::vector<T> &a, const cx<T> *tw)
{
    // as the kernels: transforms that read their input twice (inverse
    // real-DFT / DCT / DST synthesis, the extended face lines) stage their
    // lines in the tile first
    constexpr bool STAGED = reads_twice(KIND, FWD);
    std::vector<cx<T>> b0(tile_slots(AXIS, g)), b1(tile_slots(AXIS, g));
    Tile<AXIS, T> ta{b0.data(), g.L, g.RS, g.psh}, tb{b1.data(), g.L, g.RS, g.psh};
    std::vector<T> out(a.size());
    const int n = g.nl;
    auto run = [&](auto gsrc, auto put) {
        if constexpr (STAGED) {
            for (int l = 0; l < g.L; ++l)
                for (int e = 0; e < n; ++e) tile_real(ta, e, l) = gsrc(e, l);
            auto src = [&](int e, int l) -> T { return tile_real(ta, e, l); };
            tile_transform<KIND, FWD, AXIS, false, true>(0, 1, g, src, put, ta, tb, tw, NoSync());
        } else {
            tile_transform<KIND, FWD, AXIS, false, false>(0, 1, g, gsrc, put, ta, tb, tw, NoSync());
        }
    };
    if constexpr (AXIS == AX_X) {
        const long nlines = (long)ny * nz;
        for (long line0 = 0; line0 < nlines; line0 += g.L) {
            auto src = [&](int e, int l) -> T { return line0 + l < nlines ? a[(size_t)(line0 + l) * n + e] : T(0); };
            auto put = [&](int q, int l, T v) {
                if (line0 + l < nlines) out[(size_t)(line0 + l) * n + q] = v;
            };
            run(src, put);
        }
    } else {
        for (int k = 0; k < nz; ++k)
            for (int i0 = 0; i0 < nx; i0 += g.L) {
                const size_t base = (size_t)k * nx * ny;
                auto src = [&](int e, int l) -> T { return i0 + l < nx ? a[base + (size_t)e * nx + i0 + l] : T(0); };
                auto put = [&](int q, int l, T v) {
                    if (i0 + l < nx) out[base + (size_t)q * nx + i0 + l] = v;
                };
                run(src, put);
            }
    }
    a.swap(out);
}

template <typename T>
std::vector<cx<T>> tw_as(int n)
{
    std::vector<cx<double>> t = twiddles(n);
    std::vector<cx<T>> o(t.size());
    for (size_t i = 0; i < t.size(); ++i) o[i] = mk((T)t[i].re, (T)t[i].im);
    return o;
}

template <typename T>
int xform(int kind, bool fwd, int axis, int nx, int ny, int nz, std::vector<T> &a, int L = 0, int rmax = 8)
{
    const int n = axis == 0 ? nx : ny;
    XGeom g;
    if (!make_geom(g, axis == 0 ? AX_X : AX_Y, kind, n, sizeof(T), L, rmax)) return -2;
    std::vector<cx<T>> tw = tw_as<T>(fft_len(kind, n));
#define CASE(K)                                                                            \
    case K:                                                                                \
        if (axis == 0) {                                                                   \
            if (fwd) xform_k<K, true, AX_X>(g, nx, ny, nz, a, tw.data());                  \
            else xform_k<K, false, AX_X>(g, nx, ny, nz, a, tw.data());                     \
        } else {                                                                           \
            if (fwd) xform_k<K, true, AX_Y>(g, nx, ny, nz, a, tw.data());                  \
            else xform_k<K, false, AX_Y>(g, nx, ny, nz, a, tw.data());                     \
        }                                                                                  \
        break;
    switch (kind) {
        CASE(K_P) CASE(K_NN) CASE(K_DD) CASE(K_ND) CASE(K_DN) CASE(K_S1) CASE(K_C1) CASE(K_FDN) CASE(K_FND)
    }
#undef CASE
    return 0;
}

struct Setup {
    int nx, ny, nz, bc[6], kx, ky, kz;
    double dx, dy;
    std::vector<double> dzf, za, zb, zc, zaf, zcf, lamx, lamy, wc, wd, wz;
    ZArgs z;
    LapArgs la;
};

int setup(Setup &s, int nx, int ny, int nz, const int *bc, double dx, double dy, const double *dz)
{
    s.nx = nx; s.ny = ny; s.nz = nz; s.dx = dx; s.dy = dy;
    for (int i = 0; i < 6; ++i) s.bc[i] = bc[i];
    s.kx = axis_kind(bc[0], bc[1]); s.ky = axis_kind(bc[2], bc[3]); s.kz = z_kind(bc[4], bc[5]);
    if (s.kx < 0 || s.ky < 0 || s.kz < 0) return -1;
    s.dzf = z_weights(nz, bc[4], dz);
    zcoef(nz, bc[4], bc[5], std::vector<double>(dz, dz + z_widths(nz, bc[4])), s.za, s.zb, s.zc, s.zaf, s.zcf);
    s.lamx = lambdas(s.kx, nx, dx);
    s.lamy = lambdas(s.ky, ny, dy);
    const size_t N = (size_t)nx * ny * nz;
    s.wc.assign(N, 0); s.wd.assign(N, 0); s.wz.assign(N, 0);
    ZArgs &z = s.z;
    z.nx = nx; z.ny = ny; z.nz = nz;
    z.za = s.za.data(); z.zb = s.zb.data(); z.zc = s.zc.data();
    z.lamx = s.lamx.data(); z.lamy = s.lamy.data();
    z.dzf = s.dzf.data();
    long double ws = 0;
    for (int k = 0; k < nz; ++k) ws += s.dzf[k];
    z.wsum = (double)ws;
    z.scale = 1.0 / ((double)xform_scale(s.kx, nx) * (double)xform_scale(s.ky, ny));
    z.cyclic = s.kz == K_P;
    z.singular = (s.kx == K_P || s.kx == K_NN) && (s.ky == K_P || s.ky == K_NN) && (s.kz == K_P || s.kz == K_NN);
    z.wc = s.wc.data(); z.wd = s.wd.data(); z.wz = s.wz.data();
    z.removed = nullptr;
    LapArgs &la = s.la;
    la.nx = nx; la.ny = ny; la.nz = nz;
    for (int i = 0; i < 6; ++i) la.bc[i] = bc[i];
    la.idx2 = 1.0 / (dx * dx); la.idy2 = 1.0 / (dy * dy);
    la.zaf = s.zaf.data(); la.zcf = s.zcf.data();
    la.shift = 0.0;
    return 0;
}

template <typename T>
bool zsolve_part_any(Setup &s, T *data, double *removed);

// the z solve the GPU runs for this problem
template <typename T>
void zsolve_any(Setup &s, T *data, double *removed)
{
    s.z.removed = removed;
    if (!zsolve_part_any(s, data, removed))
        for (size_t col = 0; col < (size_t)s.nx * s.ny; ++col) zsolve_column(col, data, s.z);
}

template <typename T>
void solve_pass(Setup &s, std::vector<T> &a, double *removed)
{
    xform<T>(s.kx, true, 0, s.nx, s.ny, s.nz, a);
    xform<T>(s.ky, true, 1, s.nx, s.ny, s.nz, a);
    zsolve_any(s, a.data(), removed);
    xform<T>(s.ky, false, 1, s.nx, s.ny, s.nz, a);
    xform<T>(s.kx, false, 0, s.nx, s.ny, s.nz, a);
}

// the partitioned z kernel, phase by phase over all segments and columns of a
// block (CPB columns, S segments); the singular column is solved apart
template <int MMAX, bool FULL, bool CYC, bool PAD, typename T>
void zsolve_part_mm(Setup &s, T *data, double *removed, int cpb, int S)
{
    // PAD: S * MMAX levels with the kernel's padding rows in the tables
    const int nzp = PAD ? S * MMAX : s.nz;
    std::vector<double> pa(nzp), pb(nzp), pc(nzp);
    for (int k = 0; k < nzp; ++k) zpad_row(s.z, k, pa[k], pb[k], pc[k]);
    ZArgs a = s.z;
    a.za = pa.data(); a.zb = pb.data(); a.zc = pc.data();
    const size_t plane = (size_t)s.nx * s.ny;
    constexpr int NQ = CYC ? 8 : 6;
    std::vector<ZLane<MMAX, CYC>> L((size_t)S * cpb);
    std::vector<double> coef(NQ * 1024);
    auto C = [&](int q, int seg, int c) -> double & { return coef[q * 1024 + seg * cpb + c]; };
    auto lane = [&](int seg, int c) -> ZLane<MMAX, CYC> & { return L[(size_t)seg * cpb + c]; };
    for (size_t blk = 0; blk * cpb < plane; ++blk) {
        for (int w = 0; w < S; ++w)
            for (int c = 0; c < cpb; ++c) zp_load<MMAX, FULL, PAD>(lane(w, c), data, a, blk * cpb + c, zseg(nzp, S, w));
        for (int w = 0; w < S; ++w)
            for (int c = 0; c < cpb; ++c) {
                double out[NQ];
                zp_reduce<MMAX, FULL>(lane(w, c), a, zseg(nzp, S, w), out);
                for (int q = 0; q < NQ; ++q) C(q, w, c) = out[q];
            }
        for (int c = 0; c < cpb; ++c)
            zp_interface<CYC>(
                S, [&](int sg, int q) -> double & { return C(q, sg, c); },
                [&](int sg) -> double & { return C(4, sg, c); }, [&](int sg) -> double & { return C(5, sg, c); },
                [&](int sg) -> double & { return C(6 % NQ, sg, c); }, [&](int sg) -> double & { return C(7 % NQ, sg, c); });
        for (int w = 0; w < S; ++w)
            for (int c = 0; c < cpb; ++c) {
                const double xL = w > 0 ? C(5, w - 1, c) : 0.0, xR = w < S - 1 ? C(4, w + 1, c) : 0.0;
                if constexpr (CYC) {
                    const double xL2 = w > 0 ? C(7, w - 1, c) : 0.0, xR2 = w < S - 1 ? C(6, w + 1, c) : 0.0;
                    zp_finish<MMAX, FULL>(lane(w, c), a, zseg(nzp, S, w), xL, xR, xL2, xR2);
                } else {
                    zp_finish<MMAX, FULL>(lane(w, c), a, zseg(nzp, S, w), xL, xR);
                }
            }
        if constexpr (CYC) {
            for (int c = 0; c < cpb; ++c) {
                double y0, z0, yl, zl, t0, t1;
                zp_ends<MMAX, FULL>(lane(0, c), zseg(nzp, S, 0), &y0, &z0, &t0, &t1);
                zp_ends<MMAX, FULL>(lane(S - 1, c), zseg(nzp, S, S - 1), &t0, &t1, &yl, &zl);
                for (int w = 0; w < S; ++w) zp_sherman_morrison<MMAX, FULL>(lane(w, c), a, zseg(nzp, S, w), y0, z0, yl, zl);
            }
        }
        for (int w = 0; w < S; ++w)
            for (int c = 0; c < cpb; ++c) zp_store<MMAX, FULL, PAD>(lane(w, c), data, a, blk * cpb + c, zseg(nzp, S, w));
        if (a.singular && blk == 0) {
            std::vector<double> wc(s.nz), wd(s.nz);
            ZArgs as = a;
            as.removed = removed;
            zsolve_singular_ws<T>(0, data, as, wc.data(), wd.data(), 1);
        }
    }
}

// the persistent pipelined z kernel (non-periodic z, 128 < nz <= 384), phase
// by phase over the tiles of 32 columns: single-sweep reduction per segment,
// the interface of every column from both ends, the finish; padding levels
// have a zero right-hand side and are not stored
template <typename T>
void zsolve_pipe_mm(Setup &s, T *data, double *removed)
{
    constexpr int MMAX = 16, CPB = 32;
    int S = (s.nz + 15) / 16;
    S += S & 1;
    const int nzp = S * MMAX, nz = s.nz;
    std::vector<double> pa(nzp), pb(nzp), pc(nzp);
    for (int k = 0; k < nzp; ++k) zpad_row(s.z, k, pa[k], pb[k], pc[k]);
    const size_t plane = (size_t)s.nx * s.ny;
    // the singular column first (the kernel's block 0 does it before its
    // tiles), sequentially as zsolve_singular_ws
    if (s.z.singular) {
        std::vector<double> wc(nz), wd(nz);
        ZArgs as = s.z;
        as.removed = removed;
        as.za = pa.data(); as.zb = pb.data(); as.zc = pc.data();
        zsolve_singular_ws<T>(0, data, as, wc.data(), wd.data(), 1);
    }
    const size_t skip = s.z.singular ? 0 : ~(size_t)0;
    std::vector<double> coef((size_t)6 * S * CPB), r((size_t)S * CPB * MMAX), xs((size_t)S * CPB * MMAX);
    auto C = [&](int q, int sg, int c) -> double & { return coef[((size_t)sg * 6 + q) * CPB + c]; };
    for (size_t col0 = 0; col0 < plane; col0 += CPB) {
        auto own = [&](size_t col) { return col < plane && col != skip; };
        auto lam_of = [&](size_t col) { return own(col) ? s.lamx[col % s.nx] + s.lamy[col / s.nx] : -1.0; };
        auto fv_of = [&](size_t col, int k0, int q) -> double {
            const int k = k0 + q;
            return (col < plane && k < nz) ? s.z.scale * (double)data[col + plane * k] : 0.0;
        };
        for (int sg = 0; sg < S; ++sg)
            for (int c = 0; c < CPB; ++c) {
                const size_t col = col0 + c;
                auto fv = [&](int q) -> double { return fv_of(col, sg * MMAX, q); };
                double rr[MMAX], out[6];
                zp_sweep_reduce<MMAX>(fv, &pa[sg * MMAX], &pb[sg * MMAX], &pc[sg * MMAX], lam_of(col), rr, out);
                for (int q = 0; q < MMAX; ++q) r[((size_t)sg * CPB + c) * MMAX + q] = rr[q];
                for (int q = 0; q < 6; ++q) C(q, sg, c) = out[q];
            }
        for (int c = 0; c < CPB; ++c) {
            auto Cc = [&](int q, int sg) -> double & { return C(q, sg, c); };
            double y2t, g2t, y2b, g2b;
            zp_ends_forward<4>(S, false, Cc, y2t, g2t);
            zp_ends_forward<4>(S, true, Cc, y2b, g2b);
            const double pt = zp_ends_meet(y2t, g2t, y2b, g2b), pbm = zp_ends_meet(y2b, g2b, y2t, g2t);
            zp_ends_backward<4>(S, false, Cc, pt);
            zp_ends_backward<4>(S, true, Cc, pbm);
        }
        for (int sg = 0; sg < S; ++sg)
            for (int c = 0; c < CPB; ++c) {
                const size_t col = col0 + c;
                auto fv = [&](int q) -> double { return fv_of(col, sg * MMAX, q); };
                double rr[MMAX], x[MMAX];
                for (int q = 0; q < MMAX; ++q) rr[q] = r[((size_t)sg * CPB + c) * MMAX + q];
                const double xL = sg > 0 ? C(5, sg - 1, c) : 0.0, xR = sg < S - 1 ? C(4, sg + 1, c) : 0.0;
                zp_sweep_finish<MMAX>(fv, &pa[sg * MMAX], &pc[sg * MMAX], rr, xL, xR, x);
                for (int q = 0; q < MMAX; ++q) xs[((size_t)sg * CPB + c) * MMAX + q] = x[q];
            }
        for (int sg = 0; sg < S; ++sg)
            for (int c = 0; c < CPB; ++c) {
                const size_t col = col0 + c;
                if (!own(col)) continue;
                for (int q = 0; q < MMAX && sg * MMAX + q < nz; ++q)
                    data[col + plane * (sg * MMAX + q)] = (T)xs[((size_t)sg * CPB + c) * MMAX + q];
            }
    }
}

// the kernel shape the GPU launches for this nz; false when it does not apply
template <typename T>
bool zsolve_part_any(Setup &s, T *data, double *removed)
{
    if (!s.z.cyclic && s.nz > 128 && s.nz <= 384) {
        zsolve_pipe_mm(s, data, removed);
        return true;
    }
    const ZPart zp = zpart_shape(s.nz, s.z.cyclic != 0);
    if (zp.mmax == 0) return false;
    const int S = (zp.threads / 64) * (64 / zp.cpb);
    const bool full = s.nz == S * zp.mmax;
    // as the kernel launch: non-periodic z runs full segments, a ragged nz
    // padded with decoupled rows
    if (s.z.cyclic) {
        if (full) zsolve_part_mm<8, true, true, false>(s, data, removed, zp.cpb, S);
        else zsolve_part_mm<8, false, true, false>(s, data, removed, zp.cpb, S);
    } else if (zp.mmax == 8) {
        if (full) zsolve_part_mm<8, true, false, false>(s, data, removed, zp.cpb, S);
        else zsolve_part_mm<8, true, false, true>(s, data, removed, zp.cpb, S);
    } else {
        if (full) zsolve_part_mm<16, true, false, false>(s, data, removed, zp.cpb, S);
        else zsolve_part_mm<16, true, false, true>(s, data, removed, zp.cpb, S);
    }
    return true;
}

}  // namespace

extern "C" {

// The partitioned z solve (register-resident, as the GPU kernel for
// non-periodic z with nz <= 384); returns -2 when it does not apply.
int emu_zsolve_part(int nx, int ny, int nz, const int *bc, double dx, double dy, const double *dz, double *data,
                    double *removed)
{
    Setup s;
    if (setup(s, nx, ny, nz, bc, dx, dy, dz)) return -1;
    return zsolve_part_any(s, data, removed) ? 0 : -2;
}

// One transform along axis 0 (x) or 1 (y), FP64 (prec 64) or FP32 (prec 32),
// with the tile geometry (L lines, radix preference) the tuner may pick;
// L = 0 is the built-in choice.  Returns -2 when that geometry is invalid.
int emu_xform_geom(int kind, int fwd, int axis, int prec, int nx, int ny, int nz, int L, int rmax, const double *in,
                   double *out)
{
    const size_t N = (size_t)nx * ny * nz;
    int rc;
    if (prec == 64) {
        std::vector<double> a(in, in + N);
        rc = xform<double>(kind, fwd != 0, axis, nx, ny, nz, a, L, rmax);
        std::memcpy(out, a.data(), N * sizeof(double));
    } else {
        std::vector<float> a(N);
        for (size_t e = 0; e < N; ++e) a[e] = (float)in[e];
        rc = xform<float>(kind, fwd != 0, axis, nx, ny, nz, a, L, rmax);
        for (size_t e = 0; e < N; ++e) out[e] = a[e];
    }
    return rc;
}

int emu_xform(int kind, int fwd, int axis, int prec, int nx, int ny, int nz, const double *in, double *out)
{
    return emu_xform_geom(kind, fwd, axis, prec, nx, ny, nz, 0, 8, in, out);
}

// The column solves on spectral data (in place), as the z kernel does.
int emu_zsolve(int nx, int ny, int nz, const int *bc, double dx, double dy, const double *dz, double *data,
               double *removed)
{
    Setup s;
    if (setup(s, nx, ny, nz, bc, dx, dy, dz)) return -1;
    s.z.removed = removed;
    for (size_t col = 0; col < (size_t)nx * ny; ++col) zsolve_column(col, data, s.z);
    return 0;
}

// Whole solve: FP64 pipeline (max_iter < 0), or FP32 transforms with FP64
// refinement (the library's refine sequence); info = {removed mean,
// corrections, converged, last residual, history[max_iter+1]}.
int emu_solve(int nx, int ny, int nz, const int *bc, double dx, double dy, const double *dz, int max_iter,
              double tol, const double *f, double *p, double *info)
{
    Setup s;
    if (setup(s, nx, ny, nz, bc, dx, dy, dz)) return -1;
    const size_t N = (size_t)nx * ny * nz;
    double removed = 0;
    if (max_iter < 0) {
        std::vector<double> a(f, f + N);
        solve_pass<double>(s, a, &removed);
        std::memcpy(p, a.data(), N * sizeof(double));
        info[0] = removed;
        return 0;
    }
    std::vector<float> a(N);
    for (size_t e = 0; e < N; ++e) a[e] = (float)f[e];
    solve_pass<float>(s, a, nullptr);
    for (size_t e = 0; e < N; ++e) p[e] = a[e];
    const double inv_wvol = 1.0 / (s.z.wsum * nx * ny);
    if (s.z.singular) {
        double acc = 0;
        for (size_t e = 0; e < N; ++e) acc += s.dzf[e / ((size_t)nx * ny)] * f[e];
        removed = acc * inv_wvol;
    }
    info[0] = removed;
    int it = 0, conv = 0;
    double rel = -1;
    for (;; ++it) {
        double rr = 0, ff = 0, pw = 0;
        std::vector<double> r(N);
        for (int k = 0; k < nz; ++k)
            for (int j = 0; j < ny; ++j)
                for (int i = 0; i < nx; ++i) {
                    const size_t e = i + (size_t)nx * (j + (size_t)ny * k);
                    const double fv = f[e] - removed;
                    r[e] = fv - lap_point(p, i, j, k, s.la);
                    rr += r[e] * r[e];
                    ff += fv * fv;
                    pw += s.dzf[k] * p[e];
                }
        rel = ff > 0 ? std::sqrt(rr / ff) : std::sqrt(rr);
        info[4 + it] = rel;
        const double mp = s.z.singular ? pw * inv_wvol : 0.0;
        if (rel <= tol) { conv = 1; break; }
        if (it >= max_iter) break;
        for (size_t e = 0; e < N; ++e) a[e] = (float)r[e];
        solve_pass<float>(s, a, nullptr);
        for (size_t e = 0; e < N; ++e) p[e] = p[e] + (double)a[e] - mp;
    }
    info[1] = it;
    info[2] = conv;
    info[3] = rel;
    return 0;
}

}  // extern "C"

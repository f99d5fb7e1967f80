// plan.hip -- host side of the C ABI: validation, the per-axis tables of the
// eigenfunction expansion (Section 2: modified wavenumbers, transform
// twiddles, conservative z coefficients for a stretched z), device
// workspace, and the order of kernel launches of one solve.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "cans_internal.h"
#include "dense_core.h"
#include "kcommon.h"
#include "tables.h"

using namespace cans;

// Batched solves (and single solves in graph mode) run as grouped launches:
// every step of the solve is one launch per kernel variant over all the
// problems that take it (x and residual steps grouped by the x transform
// kind, y steps by the y kind, z solves by their partitioned shape), each
// block finding its problem in a table of job records.  Problems a grouped
// kernel does not cover (a dense x form, a pipelined or plain z solve, a
// check over more block partials than one block reduces) take their own
// launches at the same place of the sequence.  The sequence is captured once
// per set of (rhs, p) arrays and replayed as a single hipGraphLaunch on the
// caller's stream.
struct GroupStep {
    std::vector<GroupLaunch> grp;    // grouped launches
    std::vector<int> solo;           // problems launched on their own
};
struct FTable {
    const FJob *jobs = nullptr;
    int n = 0;
};

struct BatchGraph {
    hipGraphExec_t exec = nullptr;
    std::vector<const void *> key;   // rhs and p pointers of the tables and the captured graph
    hipStream_t cap = nullptr;
    // job tables (device), rebuilt for a new key
    void *d_tab = nullptr;
    size_t tab_bytes = 0;
    GroupStep xf, xi, yf, yi, z, rx, rn;
    // reduction records: every problem (reset), and those whose rhs mean and
    // checks one block reduces
    FTable f_all, f_mean, f_x, f_n;
    std::vector<int> fin_solo_x, fin_solo_n, mean_solo;  // the others: their own launches
    // capture branches: a step's groups touch disjoint problems and are
    // captured side by side, one stream each, forked from and joined to cap
    std::vector<hipStream_t> side;
    std::vector<hipEvent_t> ev;
};

struct cans_plan_s {
    int device = 0;
    cans_opts opts{};
    std::vector<Problem> probs;
    std::vector<void *> allocs;
    size_t bytes = 0;
    BatchGraph g;
};

namespace {

template <typename T>
int upload(cans_plan_s *pl, T **dst, const T *src, size_t count)
{
    void *p = nullptr;
    if (hipMalloc(&p, count * sizeof(T)) != hipSuccess) return CANS_ERR_ALLOC;
    pl->allocs.push_back(p);
    pl->bytes += count * sizeof(T);
    if (src && hipMemcpy(p, src, count * sizeof(T), hipMemcpyHostToDevice) != hipSuccess) return CANS_ERR_HIP;
    *dst = static_cast<T *>(p);
    return CANS_OK;
}

template <typename T>
int alloc(cans_plan_s *pl, T **dst, size_t count)
{
    return upload<T>(pl, dst, nullptr, count);
}

#define CANS_TRY(x) do { int rc_ = (x); if (rc_ != CANS_OK) return rc_; } while (0)

int validate(int nx, int ny, int nz, const int *bc, double dx, double dy, const double *dz, double shift)
{
    if (!bc || !dz || nx < 1 || ny < 1 || nz < 1) return CANS_ERR_INVALID_ARG;
    if (!(dx > 0) || !(dy > 0) || !std::isfinite(dx) || !std::isfinite(dy)) return CANS_ERR_INVALID_ARG;
    for (int i = 0; i < 6; ++i)
        if (bc[i] < 0 || bc[i] > CANS_BC_NEUMANN_FACE) return CANS_ERR_INVALID_ARG;
    // face-located pairs on x and y; on z only the Dirichlet face pair
    const int kx = axis_kind(bc[0], bc[1]), ky = axis_kind(bc[2], bc[3]);
    if (kx < 0 || ky < 0 || z_kind(bc[4], bc[5]) < 0) return CANS_ERR_INVALID_ARG;
    for (int k = 0; k < z_widths(nz, bc[4]); ++k)
        if (!(dz[k] > 0) || !std::isfinite(dz[k])) return CANS_ERR_INVALID_ARG;
    // the line the FFT sees (the line itself, or its odd / even extension for
    // a face-located Dirichlet / Neumann pair): even, up to 4096 reals (an FP64
    // line tile of two LDS buffers fits 64 KiB), half of it {2,3,5}-smooth
    const int fx = fft_len(kx, nx), fy = fft_len(ky, ny);
    if (fx < 2 || fy < 2 || fx % 2 || fy % 2 || fx > 4096 || fy > 4096) return CANS_ERR_UNSUPPORTED;
    XGeom g{};
    if (!factor(fx / 2, g) || !factor(fy / 2, g)) return CANS_ERR_UNSUPPORTED;
    // a face-located Neumann pair (DCT-I) in a problem it would make singular
    // is not handled (its compatibility weights differ from the cell form's)
    const int kz = z_kind(bc[4], bc[5]);
    if (shift == 0.0 && (kz == K_P || kz == K_NN) && has_zero_mode(kx) && has_zero_mode(ky) &&
        (kx == K_C1 || ky == K_C1))
        return CANS_ERR_UNSUPPORTED;
    if (bc[4] == CANS_BC_PERIODIC) {
        if (nz < 3) return CANS_ERR_UNSUPPORTED;
        for (int k = 1; k < nz; ++k)
            if (std::fabs(dz[k] - dz[0]) > 1e-12 * dz[0]) return CANS_ERR_UNSUPPORTED;
    }
    return CANS_OK;
}

int build_axis(cans_plan_s *pl, Axis &a, int kind, int n, double h, double shift = 0.0)
{
    a.kind = kind;
    a.n = n;
    a.h = h;
    a.s = xform_scale(kind, n);
    for (int d = 0; d < 2; ++d)
        if (!make_geom(a.gx64[d], AX_X, kind, n, 8) || !make_geom(a.gx32[d], AX_X, kind, n, 4) ||
            !make_geom(a.gy64[d], AX_Y, kind, n, 8) || !make_geom(a.gy32[d], AX_Y, kind, n, 4))
            return CANS_ERR_UNSUPPORTED;
    a.gxr32 = a.gx32[1];
    std::vector<cx<double>> t64 = twiddles(fft_len(kind, n));
    std::vector<cx<float>> t32(t64.size());
    for (size_t i = 0; i < t64.size(); ++i) t32[i] = mk((float)t64[i].re, (float)t64[i].im);
    CANS_TRY(upload(pl, &a.d_tw64, t64.data(), t64.size()));
    CANS_TRY(upload(pl, &a.d_tw32, t32.data(), t32.size()));
    std::vector<double> lam = lambdas(kind, n, h);
    for (double &v : lam) v += shift;  // the Helmholtz shift rides on one axis's eigenvalues
    CANS_TRY(upload(pl, &a.d_lam, lam.data(), n));
    return CANS_OK;
}

// bf16 hi/lo split of a long double matrix (via its FP32 value)
// bf16 hi/lo parts of a row-major n x n matrix, stored k-blocked (dense_wpos)
void split_bf16(const std::vector<long double> &W, int n, std::vector<unsigned short> &hi,
                std::vector<unsigned short> &lo)
{
    hi.resize(W.size());
    lo.resize(W.size());
    for (int q = 0; q < n; ++q)
        for (int e = 0; e < n; ++e) {
            const float x = (float)W[(size_t)q * n + e];
            const unsigned short h = to_bf16(x);
            hi[dense_wpos(n, q, e)] = h;
            lo[dense_wpos(n, q, e)] = to_bf16(x - from_bf16(h));
        }
}

int build_dense(cans_plan_s *pl, Axis &a)
{
    if (!dense_ok(a.kind, a.n)) return CANS_ERR_UNSUPPORTED;
    std::vector<unsigned short> hi, lo;
    split_bf16(dense_forward(a.kind, a.n), a.n, hi, lo);
    CANS_TRY(upload(pl, &a.d_wf_hi, hi.data(), hi.size()));
    CANS_TRY(upload(pl, &a.d_wf_lo, lo.data(), lo.size()));
    split_bf16(dense_inverse(a.kind, a.n), a.n, hi, lo);
    CANS_TRY(upload(pl, &a.d_wi_hi, hi.data(), hi.size()));
    CANS_TRY(upload(pl, &a.d_wi_lo, lo.data(), lo.size()));
    a.dense = true;
    return CANS_OK;
}

int solve_refine(const Problem &pb, const Work &w, const cans_opts &o, const double *rhs, double *p, hipStream_t s);

// Deterministic pseudo-random values in [-1, 1) (a splitmix64-style mix of
// the index): the scratch rhs of the plan-time choice of the x form.
__global__ void k_fill_unit(double *a, size_t n)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        unsigned long long h = (i + 1) * 0x9E3779B97F4A7C15ull;
        h = (h ^ (h >> 30)) * 0xBF58476D1CE4E5B9ull;
        h = (h ^ (h >> 27)) * 0x94D049BB133111EBull;
        h ^= h >> 31;
        a[i] = (double)(h >> 11) * 0x1.0p-52 - 1.0;
    }
}

// Plan-time tuning of the transform tiles: for every transform kernel the
// plan uses (x/y, forward/inverse, its precision), time the default tile and
// the candidates with a quarter .. four times the lines per tile, each with
// radix-8-first and radix-4-first plans, on a scratch field, twice each; keep
// the fastest.
// Then, for a refinement plan whose x form is left to the library (AUTO) and
// whose x axis the dense matrix-core form takes, time whole refined solves of
// a scratch rhs with the FFT and with the dense x form and keep the faster
// (the forms differ in kernel time and in the corrections they need).
int autotune(cans_plan_s *pl, Problem &pb)
{
    (void)pl;
    const size_t N = pb.npts();
    double *s64 = nullptr;
    if (hipMalloc(&s64, N * sizeof(double)) != hipSuccess) return CANS_ERR_ALLOC;
    hipStream_t st = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = CANS_OK;
    if (hipMemset(s64, 0, N * sizeof(double)) != hipSuccess || hipStreamCreate(&st) != hipSuccess ||
        hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        rc = CANS_ERR_HIP;
    if (rc == CANS_OK && pb.ws.a32 && hipMemset(pb.ws.a32, 0, N * sizeof(float)) != hipSuccess) rc = CANS_ERR_HIP;
    auto timeit = [&](auto launch) -> float {
        if (launch() != CANS_OK || launch() != CANS_OK) return 1e30f;
        (void)hipEventRecord(e0, st);
        for (int r = 0; r < 3; ++r)
            if (launch() != CANS_OK) return 1e30f;
        (void)hipEventRecord(e1, st);
        if (hipEventSynchronize(e1) != hipSuccess) return 1e30f;
        float ms = 1e30f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        return ms;
    };
    // the default tile first, then the candidates; every one is timed in two
    // passes over all of them and keeps its faster time (the first pass also
    // brings the clocks up, so the first candidates timed are not handicapped)
    auto tune = [&](XGeom &slot, int axis, const Axis &ax, int elem, auto launch) {
        std::vector<XGeom> cand{slot};
        const int L0 = slot.L;
        for (int L : {L0 / 4, L0 / 2, L0, L0 * 2, L0 * 4})
            for (int rmax : {8, 4}) {
                XGeom g;
                if (L < 1 || (L == L0 && rmax == 8) || !make_geom(g, axis, ax.kind, ax.n, elem, L, rmax)) continue;
                cand.push_back(g);
            }
        std::vector<float> t(cand.size(), 1e30f);
        for (int pass = 0; pass < 2; ++pass)
            for (size_t i = 0; i < cand.size(); ++i) {
                slot = cand[i];
                t[i] = std::min(t[i], timeit(launch));
            }
        size_t best = 0;
        for (size_t i = 1; i < cand.size(); ++i)
            if (t[i] < t[best]) best = i;
        slot = cand[best];
    };
    if (rc == CANS_OK) {
        if (pl->opts.precision == CANS_PREC_FP64) {
            tune(pb.ax.gx64[1], AX_X, pb.ax, 8, [&] { return launch_x_f64(pb, true, s64, s64, st); });
            tune(pb.ax.gx64[0], AX_X, pb.ax, 8, [&] { return launch_x_f64(pb, false, s64, s64, st); });
            tune(pb.ay.gy64[1], AX_Y, pb.ay, 8, [&] { return launch_y_f64(pb, true, s64, s64, st); });
            tune(pb.ay.gy64[0], AX_Y, pb.ay, 8, [&] { return launch_y_f64(pb, false, s64, s64, st); });
        } else {
            if (!pb.ax.dense) {
                // the forward tile is also the residual kernel's: only candidates
                // whose residual LDS fits
                tune(pb.ax.gx32[1], AX_X, pb.ax, 4,
                     [&] { return launch_x_fwd_32(pb, pb.ws, s64, pb.ws.a32, nullptr, st); });
                // the residual's fused transform: its own tile, timed as the
                // fused kernel (f = p = the scratch field)
                tune(pb.ax.gxr32, AX_X, pb.ax, 4, [&] {
                    if (resid_xfwd_lds(pb, pb.ax.gxr32) > kResidLdsMax) return (int)CANS_ERR_UNSUPPORTED;
                    return launch_resid_xfwd(pb, pb.ws, s64, s64, pb.ws.a32, pb.ws.flag, st);
                });
                tune(pb.ax.gx32[0], AX_X, pb.ax, 4,
                     [&] { return launch_x_inv_32(pb, pb.ws, pb.ws.a32, s64, false, nullptr, st); });
            }
            tune(pb.ay.gy32[1], AX_Y, pb.ay, 4, [&] { return launch_y_32(pb, true, pb.ws.a32, nullptr, st); });
            tune(pb.ay.gy32[0], AX_Y, pb.ay, 4, [&] { return launch_y_32(pb, false, pb.ws.a32, nullptr, st); });
            // (single-problem plans only: in a batch the FFT form joins its
            // kind's grouped launches, which a member timed alone does not see)
            if (pl->opts.xform_x == CANS_XFORM_AUTO && pl->probs.size() == 1 && dense_ok(pb.ax.kind, pb.nx)) {
                double *p64 = nullptr;
                if (hipMalloc(&p64, N * sizeof(double)) != hipSuccess) rc = CANS_ERR_ALLOC;
                if (rc == CANS_OK) {
                    hipLaunchKernelGGL(k_fill_unit, dim3(1024), dim3(256), 0, st, s64, N);
                    if (hipGetLastError() != hipSuccess) rc = CANS_ERR_HIP;
                }
                if (rc == CANS_OK) rc = build_dense(pl, pb.ax);
                if (rc == CANS_OK) {
                    auto solve = [&] { return solve_refine(pb, pb.ws, pl->opts, s64, p64, st); };
                    const float t_dense = timeit(solve);
                    pb.ax.dense = false;
                    const float t_fft = timeit(solve);
                    pb.ax.dense = t_dense < t_fft;
                }
                (void)hipStreamSynchronize(st);
                if (p64) (void)hipFree(p64);
            }
        }
        if (hipStreamSynchronize(st) != hipSuccess) rc = CANS_ERR_HIP;
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (st) (void)hipStreamDestroy(st);
    (void)hipFree(s64);
    return rc;
}

int build_problem(cans_plan_s *pl, Problem &pb, int nx, int ny, int nz, const int *bc, double dx, double dy,
                  const double *dz)
{
    pb.nx = nx; pb.ny = ny; pb.nz = nz;
    for (int i = 0; i < 6; ++i) pb.bc[i] = bc[i];
    pb.dzf = z_weights(nz, bc[4], dz);
    const int kx = axis_kind(bc[0], bc[1]), ky = axis_kind(bc[2], bc[3]), kz = z_kind(bc[4], bc[5]);
    CANS_TRY(build_axis(pl, pb.ax, kx, nx, dx));
    CANS_TRY(build_axis(pl, pb.ay, ky, ny, dy, pl->opts.shift));
    if (pl->opts.xform_x == CANS_XFORM_DENSE) CANS_TRY(build_dense(pl, pb.ax));
    pb.cyclic = kz == K_P;
    pb.shift = pl->opts.shift;
    pb.singular = (kx == K_P || kx == K_NN) && (ky == K_P || ky == K_NN) && (kz == K_P || kz == K_NN) &&
                  pb.shift == 0.0;
    pb.scale = 1.0 / ((double)pb.ax.s * (double)pb.ay.s);
    long double ws = 0;
    for (int k = 0; k < nz; ++k) ws += pb.dzf[k];
    pb.wsum = (double)ws;
    std::vector<double> a, b, c, af, cf;
    zcoef(nz, bc[4], bc[5], std::vector<double>(dz, dz + z_widths(nz, bc[4])), a, b, c, af, cf);
    CANS_TRY(upload(pl, &pb.d_za, a.data(), nz));
    CANS_TRY(upload(pl, &pb.d_zb, b.data(), nz));
    CANS_TRY(upload(pl, &pb.d_zc, c.data(), nz));
    CANS_TRY(upload(pl, &pb.d_zaf, af.data(), nz));
    CANS_TRY(upload(pl, &pb.d_zcf, cf.data(), nz));
    CANS_TRY(upload(pl, &pb.d_dzf, pb.dzf.data(), nz));
    CANS_TRY(plan_zpipe(pb));
    CANS_TRY(plan_resid(pb));
    // workspace of the plain elimination (nz beyond the register-resident
    // partitioned solve): multipliers and modified rhs
    const size_t N = pb.npts();
    if (zpart_shape(nz, pb.cyclic != 0).mmax == 0) {
        CANS_TRY(alloc(pl, &pb.ws.wc, N));
        CANS_TRY(alloc(pl, &pb.ws.wd, N));
        if (pb.cyclic) CANS_TRY(alloc(pl, &pb.ws.wz, N));
    }
    if (pl->opts.precision == CANS_PREC_FP32_REFINE) {
        CANS_TRY(alloc(pl, &pb.ws.a32, N));
        // block partial sums: enough for any tile shape (one row per block,
        // rows in eight slices of every plane)
        CANS_TRY(alloc(pl, &pb.ws.partials, kNP * (size_t)(pb.ny + 8) * pb.nz));
        CANS_TRY(alloc(pl, &pb.ws.sums, kNP * 256));
    }
    std::vector<double> info(I_SIZE, 0.0);
    CANS_TRY(upload(pl, &pb.ws.info, info.data(), I_SIZE));
    int zero = 0;
    CANS_TRY(upload(pl, &pb.ws.flag, &zero, 1));
    const unsigned zc2[2] = {0u, 0u};
    CANS_TRY(upload(pl, &pb.ws.zctr, zc2, 2));
    if (pl->opts.autotune) {
        CANS_TRY(autotune(pl, pb));
        // the tuning solves leave their record: start from a clean one
        if (hipMemcpy(pb.ws.info, info.data(), I_SIZE * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(pb.ws.flag, &zero, sizeof(int), hipMemcpyHostToDevice) != hipSuccess)
            return CANS_ERR_HIP;
    }
    return CANS_OK;
}

int check_opts(const cans_opts &o)
{
    if (o.precision != CANS_PREC_FP64 && o.precision != CANS_PREC_FP32_REFINE) return CANS_ERR_INVALID_ARG;
    if (o.max_iter < 0 || o.max_iter > CANS_HISTORY - 1) return CANS_ERR_INVALID_ARG;
    if (!(o.tol >= 0) || !std::isfinite(o.tol)) return CANS_ERR_INVALID_ARG;
    if (o.autotune != 0 && o.autotune != 1) return CANS_ERR_INVALID_ARG;
    if (o.graph != 0 && o.graph != 1) return CANS_ERR_INVALID_ARG;
    if (!std::isfinite(o.shift)) return CANS_ERR_INVALID_ARG;
    if (o.shift > 0) return CANS_ERR_UNSUPPORTED;  // indefinite: elimination without pivoting does not apply
    for (int m : {o.xform_x, o.xform_y})
        if (m != CANS_XFORM_AUTO && m != CANS_XFORM_FFT && m != CANS_XFORM_DENSE) return CANS_ERR_INVALID_ARG;
    // the matrix-core form exists for the x axis of the refinement path
    if (o.xform_y == CANS_XFORM_DENSE) return CANS_ERR_UNSUPPORTED;
    if (o.xform_x == CANS_XFORM_DENSE && o.precision != CANS_PREC_FP32_REFINE) return CANS_ERR_UNSUPPORTED;
    return CANS_OK;
}

void free_graph(BatchGraph &g)
{
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    g.exec = nullptr;
    if (g.cap) (void)hipStreamDestroy(g.cap);
    g.cap = nullptr;
    for (hipStream_t b : g.side) (void)hipStreamDestroy(b);
    g.side.clear();
    for (hipEvent_t e : g.ev) (void)hipEventDestroy(e);
    g.ev.clear();
    if (g.d_tab) (void)hipFree(g.d_tab);
    g.d_tab = nullptr;
    g.tab_bytes = 0;
}

void free_plan(cans_plan_s *pl)
{
    free_graph(pl->g);
    for (void *p : pl->allocs) (void)hipFree(p);
    delete pl;
}

int solve_fp64(const Problem &pb, const Work &w, const double *rhs, double *p, hipStream_t s)
{
    CANS_TRY(launch_x_f64(pb, true, rhs, p, s));
    CANS_TRY(launch_y_f64(pb, true, p, p, s));
    CANS_TRY(launch_zsolve_f64(pb, w, p, w.info + I_REMOVED, s));
    CANS_TRY(launch_y_f64(pb, false, p, p, s));
    CANS_TRY(launch_x_f64(pb, false, p, p, s));
    return CANS_OK;
}

// FP32 transforms, FP64 z elimination (the removed mean of a singular rhs
// is reduced in FP64 from the rhs itself); then up to max_iter corrections
// e = A^{-1} r with r = Pi f - L p in FP64, p <- p + e - mean(p).  Each step
// starts with a residual check; a finished flag on the device makes the
// remaining kernels return at once, so no host synchronisation is needed.
int solve_refine(const Problem &pb, const Work &w, const cans_opts &o, const double *rhs, double *p, hipStream_t s)
{
    const int *done = w.flag;
    CANS_TRY(launch_reset(pb, w, s));
    CANS_TRY(launch_x_fwd_32(pb, w, rhs, w.a32, nullptr, s));
    CANS_TRY(launch_mean_rhs(pb, w, s));
    CANS_TRY(launch_y_32(pb, true, w.a32, nullptr, s));
    CANS_TRY(launch_zsolve_32(pb, w, w.a32, nullptr, nullptr, s));
    CANS_TRY(launch_y_32(pb, false, w.a32, nullptr, s));
    CANS_TRY(launch_x_inv_32(pb, w, w.a32, p, false, nullptr, s));
    // check 0, fused with the forward x transform the first correction needs
    CANS_TRY(launch_resid_xfwd(pb, w, rhs, p, w.a32, done, s));
    CANS_TRY(launch_finalize(pb, w, resid_blocks_xfwd(pb), 0, o.max_iter, o.tol, s));
    for (int it = 1; it <= o.max_iter; ++it) {
        CANS_TRY(launch_y_32(pb, true, w.a32, done, s));
        CANS_TRY(launch_zsolve_32(pb, w, w.a32, nullptr, done, s));
        CANS_TRY(launch_y_32(pb, false, w.a32, done, s));
        CANS_TRY(launch_x_inv_32(pb, w, w.a32, p, true, done, s));
        // check `it` without a transform; only if it fails is the residual
        // formed again with its forward x transform for the next correction
        CANS_TRY(launch_resid_norm(pb, w, rhs, p, done, s));
        CANS_TRY(launch_finalize(pb, w, resid_blocks_norm(pb), it, o.max_iter, o.tol, s));
        if (it < o.max_iter) CANS_TRY(launch_resid_xfwd(pb, w, rhs, p, w.a32, done, s));
    }
    return CANS_OK;
}

int fill_info(const Problem &pb, int precision, cans_info *out)
{
    double h[I_SIZE];
    if (hipMemcpy(h, pb.ws.info, sizeof(h), hipMemcpyDeviceToHost) != hipSuccess) return CANS_ERR_HIP;
    std::memset(out, 0, sizeof(*out));
    out->removed_mean = h[I_REMOVED];
    for (int i = 0; i < CANS_HISTORY; ++i) out->history[i] = -1;
    if (precision == CANS_PREC_FP64) {
        out->iterations = 0;
        out->converged = 1;
        out->residual = -1;
        out->residual_inf = -1;
        return CANS_OK;
    }
    out->iterations = (int)h[I_ITERS];
    out->converged = (int)h[I_CONV];
    out->residual = h[I_LAST];
    out->residual_inf = h[I_LINF];
    for (int i = 0; i < CANS_HISTORY; ++i) out->history[i] = h[I_HIST + i];
    return CANS_OK;
}

// ---- the solve that allocates nothing ------------------------------------
// The per-solve buffers of cans_poisson_solve_noalloc live in this array.  In
// host code `scratch` names a host-side stand-in, not device memory: its
// device address on each GPU comes from hipGetSymbolAddress (scratch_on) and
// only that address is handed to kernels.
static __device__ __align__(256) unsigned char scratch[CANS_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char *g_scratch[kMaxDevices] = {};

// device address of the array on device `dev` (current), looked up once
int scratch_on(int dev, unsigned char **out)
{
    if (dev < 0 || dev >= kMaxDevices) return CANS_ERR_UNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return CANS_ERR_HIP;
        g_scratch[dev] = static_cast<unsigned char *>(ptr);
    }
    *out = g_scratch[dev];
    return CANS_OK;
}

// the workspace of one solve carved from `base` (256-byte aligned pieces),
// the same pieces build_problem allocates for the plan's own workspace
int carve_work(const Problem &pb, int precision, unsigned char *base, Work &w)
{
    size_t off = 0;
    auto take = [&](size_t bytes) -> unsigned char * {
        unsigned char *p = base + off;
        off += (bytes + 255) & ~(size_t)255;
        return p;
    };
    const size_t N = pb.npts();
    w = Work{};
    if (zpart_shape(pb.nz, pb.cyclic != 0).mmax == 0) {
        w.wc = reinterpret_cast<double *>(take(N * sizeof(double)));
        w.wd = reinterpret_cast<double *>(take(N * sizeof(double)));
        if (pb.cyclic) w.wz = reinterpret_cast<double *>(take(N * sizeof(double)));
    }
    if (precision == CANS_PREC_FP32_REFINE) {
        w.a32 = reinterpret_cast<float *>(take(N * sizeof(float)));
        w.partials = reinterpret_cast<double *>(take(kNP * (size_t)(pb.ny + 8) * pb.nz * sizeof(double)));
        w.sums = reinterpret_cast<double *>(take(kNP * 256 * sizeof(double)));
    }
    w.info = reinterpret_cast<double *>(take(I_SIZE * sizeof(double)));
    w.flag = reinterpret_cast<int *>(take(sizeof(int)));
    w.zctr = reinterpret_cast<unsigned *>(take(2 * sizeof(unsigned)));
    return off <= (size_t)CANS_NOALLOC_SCRATCH_BYTES ? CANS_OK : CANS_ERR_TOO_LARGE;
}

}  // namespace

namespace {

// Host side of one grouped launch while the tables are being built.
struct HostGroup {
    GroupLaunch gl;
    std::vector<unsigned char> jobs;
    std::vector<unsigned> start;
};

template <typename J>
void add_member(std::vector<HostGroup> &gs, int key, const J &job, unsigned nblk, int threads, size_t lds)
{
    HostGroup *g = nullptr;
    for (HostGroup &h : gs)
        if (h.gl.key == key) g = &h;
    if (!g) {
        gs.emplace_back();
        g = &gs.back();
        g->gl.key = key;
        g->gl.threads = 0;
    }
    g->start.push_back(g->gl.blocks);
    g->gl.blocks += (nblk + 7) / 8 * 8;  // every problem starts on a multiple of 8 (its XCD order)
    g->gl.np += 1;
    g->gl.threads = std::max(g->gl.threads, threads);
    g->gl.lds = std::max(g->gl.lds, lds);
    const unsigned char *b = reinterpret_cast<const unsigned char *>(&job);
    g->jobs.insert(g->jobs.end(), b, b + sizeof(J));
}

// One block of bytes holding every table, each at a 256-byte boundary.
struct Staging {
    std::vector<unsigned char> bytes;
    size_t put(const void *src, size_t n)
    {
        const size_t off = (bytes.size() + 255) / 256 * 256;
        bytes.resize(off + n);
        std::memcpy(bytes.data() + off, src, n);
        return off;
    }
};

XJob xjob(const Problem &pb, const void *in, void *out, const XGeom &g, const void *tw, const double *info,
          const int *done, const double *dzf, double *wsum_part)
{
    XJob j{};
    j.in = in;
    j.out = out;
    j.nlines = (long)pb.ny * pb.nz;
    j.tw = tw;
    j.info = info;
    j.done = done;
    j.dzf = dzf;
    j.wsum_part = wsum_part;
    j.ny = pb.ny;
    j.nblk = (unsigned)((j.nlines + g.L - 1) / g.L);
    j.g = g;
    return j;
}

YJob yjob(const Problem &pb, void *data, const XGeom &g, const void *tw, const int *done)
{
    YJob j{};
    j.data = data;
    j.tw = tw;
    j.done = done;
    j.nx = pb.nx;
    j.ny = pb.ny;
    j.ntx = (pb.nx + g.L - 1) / g.L;
    j.nblk = (unsigned)(j.ntx * pb.nz);
    j.g = g;
    return j;
}

// The job tables of a plan's problems for one set of (rhs, p) arrays.
int build_groups(cans_plan_s *pl, const double *const *rhs, double *const *p)
{
    BatchGraph &bg = pl->g;
    const bool refine = pl->opts.precision == CANS_PREC_FP32_REFINE;
    const size_t es = refine ? sizeof(float) : sizeof(double);
    std::vector<HostGroup> xf, xi, yf, yi, z, rx, rn;
    GroupStep *steps[] = {&bg.xf, &bg.xi, &bg.yf, &bg.yi, &bg.z, &bg.rx, &bg.rn};
    for (GroupStep *st : steps) *st = GroupStep{};
    bg.fin_solo_x.clear();
    bg.fin_solo_n.clear();
    bg.mean_solo.clear();
    std::vector<FJob> f_all, f_mean, f_x, f_n;
    struct ZMember {
        int key, threads;
        ZJob job;
    };
    std::vector<ZMember> zmem;
    for (int i = 0; i < (int)pl->probs.size(); ++i) {
        const Problem &pb = pl->probs[i];
        const Work &w = pb.ws;
        const XGeom &gxf = refine ? pb.ax.gx32[1] : pb.ax.gx64[1], &gxi = refine ? pb.ax.gx32[0] : pb.ax.gx64[0];
        const XGeom &gyf = refine ? pb.ay.gy32[1] : pb.ay.gy64[1], &gyi = refine ? pb.ay.gy32[0] : pb.ay.gy64[0];
        const void *twx = refine ? (const void *)pb.ax.d_tw32 : (const void *)pb.ax.d_tw64;
        const void *twy = refine ? (const void *)pb.ay.d_tw32 : (const void *)pb.ay.d_tw64;
        void *data = refine ? (void *)w.a32 : (void *)p[i];
        const int *done = refine ? w.flag : nullptr;
        if (pb.ax.dense) {
            bg.xf.solo.push_back(i);
            bg.xi.solo.push_back(i);
            bg.rx.solo.push_back(i);
        } else {
            const XJob jf = refine ? xjob(pb, rhs[i], w.a32, gxf, twx, nullptr, done, pb.d_dzf, w.partials)
                                   : xjob(pb, rhs[i], p[i], gxf, twx, nullptr, nullptr, nullptr, nullptr);
            const XJob ji = refine ? xjob(pb, w.a32, p[i], gxi, twx, w.info, done, nullptr, nullptr)
                                   : xjob(pb, p[i], p[i], gxi, twx, nullptr, nullptr, nullptr, nullptr);
            add_member(xf, pb.ax.kind, jf, jf.nblk, kThreads, tile_lds(AX_X, gxf, es));
            add_member(xi, pb.ax.kind, ji, ji.nblk, kThreads, tile_lds(AX_X, gxi, es));
            if (refine) {
                size_t lds = 0;
                const RJob r = rjob_xfwd(pb, w, rhs[i], p[i], w.a32, w.flag, lds);
                if (lds > kResidLdsMax) return CANS_ERR_UNSUPPORTED;
                add_member(rx, resid_group_key(pb, true), r, r.nblk, kThreads, lds);
            }
        }
        const YJob jyf = yjob(pb, data, gyf, twy, done), jyi = yjob(pb, data, gyi, twy, done);
        add_member(yf, pb.ay.kind, jyf, jyf.nblk, kThreads, tile_lds(AX_Y, gyf, es));
        add_member(yi, pb.ay.kind, jyi, jyi.nblk, kThreads, tile_lds(AX_Y, gyi, es));
        int zkey = -1, zthr = 0;
        unsigned znb = 0;
        const ZJob zj = zjob_of(pb, w, data, refine ? nullptr : w.info + I_REMOVED, done, refine, zkey, zthr, znb);
        if (zkey < 0) bg.z.solo.push_back(i);
        else zmem.push_back({zkey, zthr, zj});
        if (refine) {
            size_t lds = 0;
            const RJob r = rjob_norm(pb, w, rhs[i], p[i], w.flag, lds);
            add_member(rn, resid_group_key(pb, false), r, r.nblk, kThreads, lds);
            FJob f{};
            f.partials = w.partials;
            f.info = w.info;
            f.flag = w.flag;
            f.nb_mean = xfwd_blocks(pb);
            f.nb_xfwd = resid_blocks_xfwd(pb);
            f.nb_norm = resid_blocks_norm(pb);
            f.singular = pb.singular;
            f.inv_wvol = 1.0 / (pb.wsum * pb.nx * pb.ny);
            f_all.push_back(f);
            if (f.nb_mean <= kDirectReduce) f_mean.push_back(f); else bg.mean_solo.push_back(i);
            if (f.nb_xfwd <= kDirectReduce) f_x.push_back(f); else bg.fin_solo_x.push_back(i);
            if (f.nb_norm <= kDirectReduce) f_n.push_back(f); else bg.fin_solo_n.push_back(i);
        }
    }
    // z: blocks of each variant's deepest member; a shallower member puts
    // several column groups in a block
    for (const ZMember &m : zmem) {
        int waves = 0;
        for (const ZMember &o : zmem)
            if (o.key == m.key) waves = std::max(waves, o.threads / 64);
        ZJob j = m.job;
        j.G = zgroup_share(m.key, waves, j.S);
        j.nblk = (j.ngroups + j.G - 1) / j.G;
        add_member(z, m.key, j, j.nblk, 64 * waves, 0);
    }
    // lay the tables out in one device block
    Staging st;
    std::vector<HostGroup> *hs[] = {&xf, &xi, &yf, &yi, &z, &rx, &rn};
    std::vector<std::vector<std::pair<size_t, size_t>>> offs(7);
    for (int k = 0; k < 7; ++k)
        for (HostGroup &h : *hs[k])
            offs[k].push_back({st.put(h.jobs.data(), h.jobs.size()), st.put(h.start.data(), h.start.size() * 4)});
    std::vector<FJob> *fs[] = {&f_all, &f_mean, &f_x, &f_n};
    size_t foff[4];
    for (int k = 0; k < 4; ++k) foff[k] = st.put(fs[k]->data(), fs[k]->size() * sizeof(FJob));
    if (st.bytes.size() > bg.tab_bytes) {
        if (bg.d_tab) (void)hipFree(bg.d_tab);
        bg.d_tab = nullptr;
        bg.tab_bytes = 0;
        if (hipMalloc(&bg.d_tab, st.bytes.size()) != hipSuccess) return CANS_ERR_ALLOC;
        bg.tab_bytes = st.bytes.size();
    }
    if (!st.bytes.empty() && hipMemcpy(bg.d_tab, st.bytes.data(), st.bytes.size(), hipMemcpyHostToDevice) != hipSuccess)
        return CANS_ERR_HIP;
    unsigned char *base = static_cast<unsigned char *>(bg.d_tab);
    for (int k = 0; k < 7; ++k)
        for (size_t g = 0; g < hs[k]->size(); ++g) {
            GroupLaunch gl = (*hs[k])[g].gl;
            gl.jobs = base + offs[k][g].first;
            gl.start = reinterpret_cast<const unsigned *>(base + offs[k][g].second);
            steps[k]->grp.push_back(gl);
        }
    bg.f_all = {reinterpret_cast<const FJob *>(base + foff[0]), (int)f_all.size()};
    bg.f_mean = {reinterpret_cast<const FJob *>(base + foff[1]), (int)f_mean.size()};
    bg.f_x = {reinterpret_cast<const FJob *>(base + foff[2]), (int)f_x.size()};
    bg.f_n = {reinterpret_cast<const FJob *>(base + foff[3]), (int)f_n.size()};
    return CANS_OK;
}

// The groups of one step on their capture branches: fork from s, one side
// stream a group, join back to s (one group: on s itself).  `evi` cycles
// through the plan's events; each is waited on before it is recorded again.
template <typename F>
int each_group(const BatchGraph &bg, const GroupStep &st, hipStream_t s, size_t &evi, F launch)
{
    const size_t n = st.grp.size();
    if (n <= 1 || bg.side.size() < n || bg.ev.empty()) {
        for (const GroupLaunch &gl : st.grp) CANS_TRY(launch(gl, s));
        return CANS_OK;
    }
    hipEvent_t fork = bg.ev[evi++ % bg.ev.size()];
    if (hipEventRecord(fork, s) != hipSuccess) return CANS_ERR_HIP;
    for (size_t i = 0; i < n; ++i) {
        if (hipStreamWaitEvent(bg.side[i], fork, 0) != hipSuccess) return CANS_ERR_HIP;
        CANS_TRY(launch(st.grp[i], bg.side[i]));
    }
    for (size_t i = 0; i < n; ++i) {
        hipEvent_t join = bg.ev[evi++ % bg.ev.size()];
        if (hipEventRecord(join, bg.side[i]) != hipSuccess || hipStreamWaitEvent(s, join, 0) != hipSuccess)
            return CANS_ERR_HIP;
    }
    return CANS_OK;
}

// side streams and events for the widest step (before a capture)
int make_branches(BatchGraph &bg)
{
    size_t w = 0;
    for (const GroupStep *st : {&bg.xf, &bg.xi, &bg.yf, &bg.yi, &bg.z, &bg.rx, &bg.rn}) w = std::max(w, st->grp.size());
    while (bg.side.size() < w) {
        hipStream_t b = nullptr;
        if (hipStreamCreateWithFlags(&b, hipStreamNonBlocking) != hipSuccess) return CANS_ERR_HIP;
        bg.side.push_back(b);
    }
    while (bg.ev.size() < 16) {
        hipEvent_t e = nullptr;
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return CANS_ERR_HIP;
        bg.ev.push_back(e);
    }
    return CANS_OK;
}

// The grouped sequence of one batched solve, in the order of solve_fp64 /
// solve_refine.
int enqueue_grouped(cans_plan_s *pl, const double *const *rhs, double *const *p, hipStream_t s)
{
    const BatchGraph &bg = pl->g;
    const std::vector<Problem> &P = pl->probs;
    size_t evi = 0;
    if (pl->opts.precision == CANS_PREC_FP64) {
        CANS_TRY(each_group(bg, bg.xf, s, evi,
                            [](const GroupLaunch &g, hipStream_t b) { return launch_x_f64_grp(g, true, b); }));
        CANS_TRY(each_group(bg, bg.yf, s, evi,
                            [](const GroupLaunch &g, hipStream_t b) { return launch_y_f64_grp(g, true, b); }));
        CANS_TRY(each_group(bg, bg.z, s, evi,
                            [](const GroupLaunch &g, hipStream_t b) { return launch_zsolve_grp(g, false, b); }));
        for (int i : bg.z.solo) CANS_TRY(launch_zsolve_f64(P[i], P[i].ws, p[i], P[i].ws.info + I_REMOVED, s));
        CANS_TRY(each_group(bg, bg.yi, s, evi,
                            [](const GroupLaunch &g, hipStream_t b) { return launch_y_f64_grp(g, false, b); }));
        CANS_TRY(each_group(bg, bg.xi, s, evi,
                            [](const GroupLaunch &g, hipStream_t b) { return launch_x_f64_grp(g, false, b); }));
        return CANS_OK;
    }
    const cans_opts &o = pl->opts;
    auto ystep = [&](bool fwd) {
        return each_group(bg, fwd ? bg.yf : bg.yi, s, evi,
                          [&](const GroupLaunch &g, hipStream_t b) { return launch_y_32_grp(g, fwd, b); });
    };
    auto zstep = [&](bool first) {
        CANS_TRY(each_group(bg, bg.z, s, evi,
                            [](const GroupLaunch &g, hipStream_t b) { return launch_zsolve_grp(g, true, b); }));
        for (int i : bg.z.solo)
            CANS_TRY(launch_zsolve_32(P[i], P[i].ws, P[i].ws.a32, nullptr, first ? nullptr : P[i].ws.flag, s));
        return (int)CANS_OK;
    };
    auto xinv = [&](bool update) {
        CANS_TRY(each_group(bg, bg.xi, s, evi,
                            [&](const GroupLaunch &g, hipStream_t b) { return launch_x_inv_32_grp(g, update, b); }));
        for (int i : bg.xi.solo)
            CANS_TRY(launch_x_inv_32(P[i], P[i].ws, P[i].ws.a32, p[i], update, update ? P[i].ws.flag : nullptr, s));
        return (int)CANS_OK;
    };
    auto rxstep = [&]() {
        CANS_TRY(each_group(bg, bg.rx, s, evi,
                            [](const GroupLaunch &g, hipStream_t b) { return launch_resid_xfwd_grp(g, b); }));
        for (int i : bg.rx.solo) CANS_TRY(launch_resid_xfwd(P[i], P[i].ws, rhs[i], p[i], P[i].ws.a32, P[i].ws.flag, s));
        return (int)CANS_OK;
    };
    auto check = [&](int which, int it) {
        const FTable &t = which == 0 ? bg.f_x : bg.f_n;
        if (t.n) CANS_TRY(launch_finalize_grp(t.jobs, t.n, which, it, o.max_iter, o.tol, s));
        for (int i : which == 0 ? bg.fin_solo_x : bg.fin_solo_n)
            CANS_TRY(launch_finalize(P[i], P[i].ws, which == 0 ? resid_blocks_xfwd(P[i]) : resid_blocks_norm(P[i]), it,
                                     o.max_iter, o.tol, s));
        return (int)CANS_OK;
    };
    CANS_TRY(launch_reset_grp(bg.f_all.jobs, bg.f_all.n, s));
    CANS_TRY(each_group(bg, bg.xf, s, evi,
                        [](const GroupLaunch &g, hipStream_t b) { return launch_x_fwd_32_grp(g, b); }));
    for (int i : bg.xf.solo) CANS_TRY(launch_x_fwd_32(P[i], P[i].ws, rhs[i], P[i].ws.a32, nullptr, s));
    if (bg.f_mean.n) CANS_TRY(launch_mean_rhs_grp(bg.f_mean.jobs, bg.f_mean.n, s));
    for (int i : bg.mean_solo) CANS_TRY(launch_mean_rhs(P[i], P[i].ws, s));
    CANS_TRY(ystep(true));
    CANS_TRY(zstep(true));
    CANS_TRY(ystep(false));
    CANS_TRY(xinv(false));
    // check 0, fused with the forward x transform the first correction needs
    CANS_TRY(rxstep());
    CANS_TRY(check(0, 0));
    for (int it = 1; it <= o.max_iter; ++it) {
        CANS_TRY(ystep(true));
        CANS_TRY(zstep(false));
        CANS_TRY(ystep(false));
        CANS_TRY(xinv(true));
        CANS_TRY(each_group(bg, bg.rn, s, evi,
                            [](const GroupLaunch &g, hipStream_t b) { return launch_resid_norm_grp(g, b); }));
        CANS_TRY(check(1, it));
        if (it < o.max_iter) CANS_TRY(rxstep());
    }
    return CANS_OK;
}

}  // namespace

extern "C" {

void cans_default_opts(cans_opts *o)
{
    if (!o) return;
    o->precision = CANS_PREC_FP64;
    o->xform_x = CANS_XFORM_AUTO;
    o->xform_y = CANS_XFORM_AUTO;
    o->tol = 1e-10;
    o->max_iter = 4;
    o->autotune = 0;
    o->graph = 0;
    o->shift = 0.0;
}

const char *cans_status_string(int code)
{
    switch (code) {
    case CANS_OK: return "ok";
    case CANS_ERR_INVALID_ARG: return "invalid argument";
    case CANS_ERR_UNSUPPORTED: return "unsupported problem";
    case CANS_ERR_ALLOC: return "allocation failed";
    case CANS_ERR_HIP: return "HIP runtime error";
    case CANS_ERR_ALIAS: return "rhs and p alias";
    case CANS_ERR_TOO_LARGE: return "problem exceeds the fixed scratch of the no-allocation solve";
    default: return "unknown status";
    }
}

int cans_poisson_plan_ex(cans_plan_t *out, int nx, int ny, int nz, const int bc[6], double dx, double dy,
                         const double *dz, const cans_opts *opts)
{
    if (!out) return CANS_ERR_INVALID_ARG;
    *out = nullptr;
    cans_desc d;
    d.nx = nx; d.ny = ny; d.nz = nz;
    if (bc) for (int i = 0; i < 6; ++i) d.bc[i] = bc[i];
    d.dx = dx; d.dy = dy; d.dz = dz;
    if (!bc) return CANS_ERR_INVALID_ARG;
    return cans_poisson_plan_batched(out, 1, &d, opts);
}

int cans_poisson_plan(cans_plan_t *out, int nx, int ny, int nz, const int bc[6], double dx, double dy,
                      const double *dz)
{
    return cans_poisson_plan_ex(out, nx, ny, nz, bc, dx, dy, dz, nullptr);
}

int cans_poisson_plan_batched(cans_plan_t *out, int count, const cans_desc *descs, const cans_opts *opts)
{
    if (!out || count < 1 || !descs) return CANS_ERR_INVALID_ARG;
    *out = nullptr;
    cans_opts o;
    cans_default_opts(&o);
    if (opts) o = *opts;
    CANS_TRY(check_opts(o));
    for (int i = 0; i < count; ++i)
        CANS_TRY(validate(descs[i].nx, descs[i].ny, descs[i].nz, descs[i].bc, descs[i].dx, descs[i].dy,
                          descs[i].dz, o.shift));
    cans_plan_s *pl = new (std::nothrow) cans_plan_s();
    if (!pl) return CANS_ERR_ALLOC;
    pl->opts = o;
    if (hipGetDevice(&pl->device) != hipSuccess) { delete pl; return CANS_ERR_HIP; }
    pl->probs.resize(count);
    for (int i = 0; i < count; ++i) {
        const cans_desc &d = descs[i];
        int rc = build_problem(pl, pl->probs[i], d.nx, d.ny, d.nz, d.bc, d.dx, d.dy, d.dz);
        if (rc != CANS_OK) { free_plan(pl); return rc; }
    }
    *out = pl;
    return CANS_OK;
}

int cans_poisson_solve(cans_plan_t plan, const double *rhs, double *p, hipStream_t stream)
{
    if (!plan || !rhs || !p || plan->probs.size() != 1) return CANS_ERR_INVALID_ARG;
    if (plan->opts.graph) return cans_poisson_solve_batched(plan, &rhs, &p, stream);
    const Problem &pb = plan->probs[0];
    if (plan->opts.precision == CANS_PREC_FP64) return solve_fp64(pb, pb.ws, rhs, p, stream);
    if ((const void *)rhs == (const void *)p) return CANS_ERR_ALIAS;
    return solve_refine(pb, pb.ws, plan->opts, rhs, p, stream);
}

int cans_poisson_solve_noalloc(cans_plan_t plan, const double *rhs, double *p, hipStream_t stream)
{
    if (!plan || !rhs || !p || plan->probs.size() != 1) return CANS_ERR_INVALID_ARG;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return CANS_ERR_HIP;
    if (dev != plan->device) return CANS_ERR_INVALID_ARG;
    const Problem &pb = plan->probs[0];
    const int prec = plan->opts.precision;
    if (prec != CANS_PREC_FP64 && (const void *)rhs == (const void *)p) return CANS_ERR_ALIAS;
    unsigned char *base = nullptr;
    CANS_TRY(scratch_on(dev, &base));
    Work w;
    CANS_TRY(carve_work(pb, prec, base, w));
    // the array keeps the previous call's contents: clear what must start at zero
    CANS_TRY(launch_clear_work(w, stream));
    CANS_TRY(prec == CANS_PREC_FP64 ? solve_fp64(pb, w, rhs, p, stream) : solve_refine(pb, w, plan->opts, rhs, p, stream));
    return launch_copy_info(w.info, pb.ws.info, stream);
}

int cans_poisson_project_ex(cans_plan_t plan, double *u, double *v, double *w, double *p, double gdt, double alpha,
                            double nu, double *dt_max, hipStream_t stream)
{
    if (!plan || !u || !v || !w || !p || plan->probs.size() != 1) return CANS_ERR_INVALID_ARG;
    if (!(gdt > 0) || !std::isfinite(gdt)) return CANS_ERR_INVALID_ARG;
    if (!(alpha >= 0) || !std::isfinite(alpha) || !(nu >= 0) || !std::isfinite(nu)) return CANS_ERR_INVALID_ARG;
    if (plan->opts.precision != CANS_PREC_FP64 || plan->opts.shift != 0.0) return CANS_ERR_UNSUPPORTED;
    Problem &pb = plan->probs[0];
    for (int a = 0; a < 3; ++a)
        if (pb.bc[2 * a] != pb.bc[2 * a + 1] ||
            (pb.bc[2 * a] != CANS_BC_PERIODIC && pb.bc[2 * a] != CANS_BC_NEUMANN))
            return CANS_ERR_UNSUPPORTED;
    const void *f[5] = {u, v, w, p, dt_max};
    for (int a = 0; a < 5; ++a)
        for (int b = a + 1; b < 5; ++b)
            if (f[a] && f[a] == f[b]) return CANS_ERR_ALIAS;
    if (!pb.phi) {
        // first use: the potential field, the z centre distances across each
        // +z face (and their inverses, 0 on a wall face) and the block maxima
        // of the time-step rates
        const int nz = pb.nz;
        std::vector<double> zgc(nz, 0.0), dzc(nz, 0.0);
        for (int k = 0; k + 1 < nz; ++k) {
            dzc[k] = 0.5 * (pb.dzf[k] + pb.dzf[k + 1]);
            zgc[k] = 2.0 / (pb.dzf[k] + pb.dzf[k + 1]);
        }
        dzc[nz - 1] = pb.cyclic ? 0.5 * (pb.dzf[nz - 1] + pb.dzf[0]) : pb.dzf[nz - 1];
        if (pb.cyclic) zgc[nz - 1] = 2.0 / (pb.dzf[nz - 1] + pb.dzf[0]);
        CANS_TRY(upload(plan, &pb.d_zgc, zgc.data(), nz));
        CANS_TRY(upload(plan, &pb.d_dzc, dzc.data(), nz));
        CANS_TRY(alloc(plan, &pb.dt_part, (size_t)dt_blocks(pb)));
        CANS_TRY(alloc(plan, &pb.phi, pb.npts()));
    }
    CANS_TRY(launch_div_xfwd(pb, u, v, w, gdt, pb.phi, stream));
    CANS_TRY(launch_y_f64(pb, true, pb.phi, pb.phi, stream));
    CANS_TRY(launch_zsolve_f64(pb, pb.ws, pb.phi, pb.ws.info + I_REMOVED, stream));
    CANS_TRY(launch_y_f64(pb, false, pb.phi, pb.phi, stream));
    CANS_TRY(launch_x_f64(pb, false, pb.phi, pb.phi, stream));
    CANS_TRY(launch_project_correct(pb, u, v, w, p, pb.phi, gdt, alpha, stream));
    if (dt_max) CANS_TRY(launch_max_dt(pb, u, v, w, nu, dt_max, stream));
    return CANS_OK;
}

int cans_poisson_project(cans_plan_t plan, double *u, double *v, double *w, double *p, double gdt,
                         hipStream_t stream)
{
    return cans_poisson_project_ex(plan, u, v, w, p, gdt, 0.0, 0.0, nullptr, stream);
}

int cans_poisson_solve_batched(cans_plan_t plan, const double *const *rhs, double *const *p, hipStream_t stream)
{
    if (!plan || !rhs || !p) return CANS_ERR_INVALID_ARG;
    const size_t n = plan->probs.size();
    std::vector<const void *> key(2 * n);
    for (size_t i = 0; i < n; ++i) {
        if (!rhs[i] || !p[i]) return CANS_ERR_INVALID_ARG;
        if (plan->opts.precision != CANS_PREC_FP64 && (const void *)rhs[i] == (const void *)p[i])
            return CANS_ERR_ALIAS;
        key[2 * i] = rhs[i];
        key[2 * i + 1] = p[i];
    }
    BatchGraph &g = plan->g;
    if (!g.exec || g.key != key) {
        // new arrays: rebuild the job tables (after the work that may still
        // read the old ones) and capture the grouped sequence once
        if (g.exec) {
            if (hipStreamSynchronize(stream) != hipSuccess) return CANS_ERR_HIP;
            (void)hipGraphExecDestroy(g.exec);
            g.exec = nullptr;
        }
        g.key.clear();
        if (!g.cap && hipStreamCreateWithFlags(&g.cap, hipStreamNonBlocking) != hipSuccess) return CANS_ERR_HIP;
        CANS_TRY(build_groups(plan, rhs, p));
        CANS_TRY(make_branches(g));
        if (hipStreamBeginCapture(g.cap, hipStreamCaptureModeThreadLocal) != hipSuccess) return CANS_ERR_HIP;
        const int rc = enqueue_grouped(plan, rhs, p, g.cap);
        hipGraph_t graph = nullptr;
        const hipError_t ec = hipStreamEndCapture(g.cap, &graph);
        if (rc != CANS_OK || ec != hipSuccess) {
            if (graph) (void)hipGraphDestroy(graph);
            return rc != CANS_OK ? rc : CANS_ERR_HIP;
        }
        const hipError_t ei = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (ei != hipSuccess) {
            g.exec = nullptr;
            return CANS_ERR_HIP;
        }
        g.key = key;
    }
    return hipGraphLaunch(g.exec, stream) == hipSuccess ? CANS_OK : CANS_ERR_HIP;
}

int cans_poisson_get_info(cans_plan_t plan, cans_info *out)
{
    if (!plan || !out) return CANS_ERR_INVALID_ARG;
    return fill_info(plan->probs[0], plan->opts.precision, out);
}

int cans_poisson_get_info_batched(cans_plan_t plan, int index, cans_info *out)
{
    if (!plan || !out || index < 0 || index >= (int)plan->probs.size()) return CANS_ERR_INVALID_ARG;
    return fill_info(plan->probs[index], plan->opts.precision, out);
}

size_t cans_poisson_workspace_bytes(cans_plan_t plan) { return plan ? plan->bytes : 0; }

int cans_poisson_xform_mode(cans_plan_t plan, int axis)
{
    if (!plan || plan->probs.size() != 1 || (axis != 0 && axis != 1)) return CANS_ERR_INVALID_ARG;
    return axis == 0 && plan->probs[0].ax.dense ? CANS_XFORM_DENSE : CANS_XFORM_FFT;
}

int cans_poisson_debug_stage(cans_plan_t plan, int stage, const double *in, double *out, hipStream_t stream)
{
    if (!plan || plan->probs.size() != 1) return CANS_ERR_INVALID_ARG;
    const Problem &pb = plan->probs[0];
    if (plan->opts.precision == CANS_PREC_FP32_REFINE) {
        // single kernels of the refinement path on the plan's FP32 field
        switch (stage) {
        case 1: return in ? launch_x_fwd_32(pb, pb.ws, in, pb.ws.a32, nullptr, stream) : CANS_ERR_INVALID_ARG;
        case 2: return launch_y_32(pb, true, pb.ws.a32, nullptr, stream);
        case 3: return launch_zsolve_32(pb, pb.ws, pb.ws.a32, nullptr, nullptr, stream);
        case 4: return launch_y_32(pb, false, pb.ws.a32, nullptr, stream);
        case 5: return out ? launch_x_inv_32(pb, pb.ws, pb.ws.a32, out, false, nullptr, stream) : CANS_ERR_INVALID_ARG;
        case 0: return launch_reset(pb, pb.ws, stream);
        case 6:
            if (!in || !out) return CANS_ERR_INVALID_ARG;
            return launch_resid_xfwd(pb, pb.ws, in, out, pb.ws.a32, pb.ws.flag, stream);
        case 7: return out ? launch_x_inv_32(pb, pb.ws, pb.ws.a32, out, true, nullptr, stream) : CANS_ERR_INVALID_ARG;
        case 8:
            if (!in || !out) return CANS_ERR_INVALID_ARG;
            return launch_resid_norm(pb, pb.ws, in, out, pb.ws.flag, stream);
        default: return CANS_ERR_INVALID_ARG;
        }
    }
    if (!in || !out) return CANS_ERR_INVALID_ARG;
    switch (stage) {
    case 1: return launch_x_f64(pb, true, in, out, stream);
    case 2: return launch_y_f64(pb, true, in, out, stream);
    case 3:
        if (in != out && hipMemcpyAsync(out, in, pb.npts() * sizeof(double), hipMemcpyDeviceToDevice, stream) !=
                             hipSuccess)
            return CANS_ERR_HIP;
        return launch_zsolve_f64(pb, pb.ws, out, pb.ws.info + I_REMOVED, stream);
    case 4: return launch_y_f64(pb, false, in, out, stream);
    case 5: return launch_x_f64(pb, false, in, out, stream);
    default: return CANS_ERR_INVALID_ARG;
    }
}

void cans_poisson_destroy(cans_plan_t plan)
{
    if (plan) free_plan(plan);
}

}  // extern "C"

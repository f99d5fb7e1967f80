// cans_internal.h -- plan layout and kernel launchers shared by the host
// plan code and the HIP kernels (not part of the public ABI).
#pragma once

#include <vector>

#include "../../include/cans_poisson.h"
#include "zsolve_core.h"

namespace cans {

// device-side info record of one problem (doubles)
enum InfoSlot {
    I_REMOVED = 0,   // removed weighted mean of the rhs (singular problems)
    I_MEANP = 1,     // weighted mean of p measured by the last residual pass
    I_ITERS = 2,     // corrections applied
    I_CONV = 3,      // 1 when the residual test passed
    I_LAST = 4,      // last relative residual
    I_HIST = 5,      // CANS_HISTORY entries
    I_LINF = I_HIST + CANS_HISTORY,  // last residual in the max norm
    I_SIZE = I_LINF + 1
};

// values per block partial of the reductions: sum r^2, sum (Pi f)^2,
// sum dzf p, max |r|, max |Pi f| (the first pass uses entry 0 only)
constexpr int kNP = 5;

constexpr int kThreads = 256;  // threads per block of the transform kernels

struct Axis {
    int kind = 0;
    int n = 0;
    double h = 1;
    int s = 1;                 // B T = s I
    // tile geometry as an x or a y transform, FP64 / FP32, [0] inverse [1] forward
    XGeom gx64[2]{}, gx32[2]{};
    XGeom gy64[2]{}, gy32[2]{};
    XGeom gxr32{};             // the forward FP32 x tile of the kernel fused with the residual
    double *d_lam = nullptr;   // mu(q)/h^2 in the transform's row order
    cx<double> *d_tw64 = nullptr;
    cx<float> *d_tw32 = nullptr;
    // dense (matrix-core) form: bf16 hi/lo of the forward and inverse matrices
    bool dense = false;
    unsigned short *d_wf_hi = nullptr, *d_wf_lo = nullptr, *d_wi_hi = nullptr, *d_wi_lo = nullptr;
};

// Per-solve mutable device memory of one problem: the plan's own (allocated
// when the plan is built), or carved from the library's static scratch array
// by the entry point that allocates nothing.
struct Work {
    float *a32 = nullptr;          // FP32 spectral field (refine mode)
    double *partials = nullptr;    // block partial sums of the reductions
    double *sums = nullptr;        // first-level sums of the partials (256 records)
    double *info = nullptr;        // info record, I_SIZE doubles
    int *flag = nullptr;           // [0] refinement finished
    double *wc = nullptr, *wd = nullptr, *wz = nullptr;  // plain elimination (deep or periodic z)
    unsigned *zctr = nullptr;      // pipelined z solve: tiles claimed, blocks finished (zero between launches)
};

// Launch shape of the persistent, pipelined z solve (k_zsolve_pipe), chosen
// when the plan is built; off when the problem does not fit it.
constexpr int kPipeCols = 32;      // columns per tile
constexpr int kPipeThreads = 768;  // largest block (24 segments of 16 levels)
struct PipePlan {
    bool on = false;
    bool db = false;   // two tile buffers in LDS
    int threads = 0, grid = 0, ntiles = 0;
    size_t lds = 0;
};

struct Problem {
    int nx = 0, ny = 0, nz = 0;
    int bc[6] = {0, 0, 0, 0, 0, 0};
    Axis ax, ay;
    std::vector<double> dzf;
    double wsum = 0;
    int cyclic = 0, singular = 0;
    double shift = 0;              // Helmholtz shift s of (L_h + s) p = f
    double scale = 1;
    double *d_za = nullptr, *d_zb = nullptr, *d_zc = nullptr;
    double *d_zaf = nullptr, *d_zcf = nullptr, *d_dzf = nullptr;
    Work ws;                       // the plan's own workspace
    PipePlan zpipe32, zpipe64;     // pipelined z solve for FP32 / FP64 data
    // projection step (allocated at its first use)
    double *phi = nullptr;         // the potential Phi (FP64 field)
    double *d_zgc = nullptr;       // 1/dzc_k across the +z face of level k, 0 on a wall face
    double *d_dzc = nullptr;       // dzc_k across the +z face of level k (the mirror cell's at a wall)
    double *dt_part = nullptr;     // block maxima of the time-step rates
    size_t npts() const { return (size_t)nx * ny * nz; }
};

// ---- grouped launches of a batch -------------------------------------------
// A batched plan runs each step of the solve as one launch per kernel variant
// over all the problems that take it (the same transform kind, or the same z
// solve shape).  Each block finds its problem in `start` (first block of each
// problem, multiples of 8) and reads the problem's job record.
struct XJob {            // x transform of one problem
    const void *in;
    void *out;
    long nlines;
    const void *tw;
    const double *info;
    const int *done;
    const double *dzf;
    double *wsum_part;
    int ny;
    unsigned nblk;       // blocks of this problem (the launch may give it a few more, which return)
    XGeom g;
};
struct YJob {            // y transform of one problem, in place
    void *data;
    const void *tw;
    const int *done;
    int nx, ny, ntx;
    unsigned nblk;
    XGeom g;
};
struct ZJob {            // partitioned z solve of one problem
    void *data;
    const int *done;
    int S;               // its segments
    int G;               // its column groups a block (the launch's blocks may hold more waves)
    unsigned ngroups;    // its column groups
    unsigned nblk;       // ceil(ngroups / G)
    ZArgs a;
};
struct RJob {            // residual pass of one problem (fused with the x transform, or norms only)
    const double *f, *p;
    float *out;
    const void *tw;
    const double *dzf, *info;
    double *partials;
    const int *done;
    int H, bpp, L, rows_off;
    unsigned nblk;
    LapArgs la;
    XGeom g;
};
struct FJob {            // per-problem reductions: reset, rhs mean, convergence check
    double *partials;
    double *info;
    int *flag;
    int nb_mean, nb_xfwd, nb_norm;   // partials of the first x transform, the fused and the norm pass
    int singular;
    double inv_wvol;
};

// One grouped launch: its device tables and shape.
struct GroupLaunch {
    int key = 0;                 // kernel variant (transform kind, or z shape code)
    int np = 0;                  // problems
    unsigned blocks = 0;         // grid
    int threads = kThreads;
    size_t lds = 0;              // dynamic LDS: the largest member's
    const void *jobs = nullptr;  // device job records
    const unsigned *start = nullptr;
};

int launch_x_fwd_32_grp(const GroupLaunch &gl, hipStream_t s);
int launch_x_inv_32_grp(const GroupLaunch &gl, bool update, hipStream_t s);
int launch_x_f64_grp(const GroupLaunch &gl, bool fwd, hipStream_t s);
int launch_y_32_grp(const GroupLaunch &gl, bool fwd, hipStream_t s);
int launch_y_f64_grp(const GroupLaunch &gl, bool fwd, hipStream_t s);
int launch_zsolve_grp(const GroupLaunch &gl, bool fp32, hipStream_t s);
int launch_resid_xfwd_grp(const GroupLaunch &gl, hipStream_t s);
int launch_resid_norm_grp(const GroupLaunch &gl, hipStream_t s);
int launch_reset_grp(const FJob *jobs, int np, hipStream_t s);
int launch_mean_rhs_grp(const FJob *jobs, int np, hipStream_t s);
int launch_finalize_grp(const FJob *jobs, int np, int which, int check, int max_iter, double tol, hipStream_t s);
// job records (and, for z, the variant key and block shape; key < 0: this
// problem's z solve is not a partitioned one and runs on its own)
ZJob zjob_of(const Problem &pb, const Work &w, void *data, double *removed, const int *done, bool fp32, int &key,
             int &threads, unsigned &nblk);
int zgroup_share(int key, int waves, int S);
int resid_group_key(const Problem &pb, bool fused);
RJob rjob_xfwd(const Problem &pb, const Work &w, const double *f, const double *p, float *out, const int *done,
               size_t &lds);
RJob rjob_norm(const Problem &pb, const Work &w, const double *f, const double *p, const int *done, size_t &lds);
// largest number of block partials a grouped check reduces in its one block
constexpr int kDirectReduce = 4096;

// ---- launchers (k_xform.hip, k_zsolve.hip, k_resid.hip, k_project.hip) -----
// x transform of nlines contiguous lines; dir 1 forward, 0 inverse.
// Tin/Tout: double or float; epi 0 store, 1 update p += v - info[I_MEANP].
int launch_x_f64(const Problem &pb, bool fwd, const double *in, double *out, hipStream_t s);
int launch_y_f64(const Problem &pb, bool fwd, const double *in, double *out, hipStream_t s);
// (also leaves FP64 block sums of dzf*in in w.partials for launch_mean_rhs)
int launch_x_fwd_32(const Problem &pb, const Work &w, const double *in, float *out, const int *done, hipStream_t s);
int launch_y_32(const Problem &pb, bool fwd, float *data, const int *done, hipStream_t s);
int launch_x_inv_32(const Problem &pb, const Work &w, const float *in, double *p, bool update, const int *done,
                    hipStream_t s);
int launch_zsolve_f64(const Problem &pb, const Work &w, double *data, double *removed, hipStream_t s);
// choose the pipelined z-solve shapes of a problem (plan time)
int plan_zpipe(Problem &pb);
int launch_zsolve_32(const Problem &pb, const Work &w, float *data, double *removed, const int *done, hipStream_t s);
// refinement: residual fused with the forward x transform (FP32 out), and the
// residual norm alone; then the reduction that decides convergence.
int launch_resid_xfwd(const Problem &pb, const Work &w, const double *f, const double *p, float *out,
                      const int *done, hipStream_t s);
int launch_resid_norm(const Problem &pb, const Work &w, const double *f, const double *p, const int *done,
                      hipStream_t s);
// nblk: the block partials the preceding residual kernel wrote
int launch_finalize(const Problem &pb, const Work &w, int nblk, int check, int max_iter, double tol, hipStream_t s);
int launch_reset(const Problem &pb, const Work &w, hipStream_t s);
// zero a workspace's info record, flag and z-solve counters (a kernel, so the
// sequence stays capturable); copy an info record to another
int launch_clear_work(const Work &w, hipStream_t s);
int launch_copy_info(const double *src, double *dst, hipStream_t s);
int launch_mean_rhs(const Problem &pb, const Work &w, hipStream_t s);

// block partials written by launch_resid_xfwd / launch_resid_norm (at most
// kNP (ny + 8) nz doubles); plan_resid: their LDS limits (plan time)
int resid_blocks_xfwd(const Problem &pb);
int resid_blocks_norm(const Problem &pb);
int plan_resid(const Problem &pb);
// LDS bytes the residual+transform kernel needs with x tile g; the largest
// the plan allows it (tile candidates beyond it are not used)
size_t resid_xfwd_lds(const Problem &pb, const XGeom &g);
constexpr size_t kResidLdsMax = 156 * 1024;

// projection step: D u / gdt fused into the forward x transform (FP64, into
// out), and the correction u -= gdt G phi, p += phi - alpha L_h phi
int launch_div_xfwd(const Problem &pb, const double *u, const double *v, const double *w, double gdt, double *out,
                    hipStream_t s);
int launch_project_correct(const Problem &pb, double *u, double *v, double *w, double *p, const double *phi,
                           double gdt, double alpha, hipStream_t s);
// time-step bound of eq. (dt) on a staggered velocity into dt (device, one
// double); pb.dt_part holds dt_blocks(pb) block maxima
int dt_blocks(const Problem &pb);
int launch_max_dt(const Problem &pb, const double *u, const double *v, const double *w, double nu, double *dt,
                  hipStream_t s);

}  // namespace cans

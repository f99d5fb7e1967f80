// k_zsolve.hip -- the FP64 z solve of the column systems of eq. (poi_reduced) (Section 2) and
// its launchers.
#include "kcommon.h"

namespace cans {

template <typename T>
__global__ __launch_bounds__(256) void k_zsolve(T *data, ZArgs a, const int *__restrict__ done)
{
    if (done && *done) return;
    const size_t col = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (col >= (size_t)a.nx * a.ny) return;
    zsolve_column(col, data, a);
}

static ZArgs zargs(const Problem &pb, const Work &w, double *removed);

// Partitioned column solve: CPB adjacent columns per block (64 or 32), z split
// into S segments of at most MMAX levels held in registers; a wave holds
// 64/CPB segments of the same columns (see zsolve_core.h).
template <typename T, int MMAX, int CPB, int NTMAX, bool FULL, bool CYC, bool PAD = false>
__global__ __launch_bounds__(NTMAX) void k_zsolve_part(T *data, ZArgs ag, const int *__restrict__ done)
{
    if (done && *done) return;
    constexpr int NQ = CYC ? 8 : 6;  // interface coefficients per segment
    __shared__ double coef[NQ * 1024];
    __shared__ double zabc[3 * 512];  // the z coefficients, staged once per block
    __shared__ double ends[CYC ? 4 * 64 : 1];  // CYC: first/last values per column
    constexpr int SPW = 64 / CPB;  // segments per wave
    // PAD: S * MMAX levels (<= 512 for every launched shape), padding rows
    // beyond nz
    const int nzp = PAD ? (int)(blockDim.x >> 6) * SPW * MMAX : ag.nz;
    for (int i = threadIdx.x; i < nzp; i += blockDim.x)
        zpad_row(ag, i, zabc[i], zabc[512 + i], zabc[1024 + i]);
    ZArgs a = ag;
    a.za = zabc;
    a.zb = zabc + 512;
    a.zc = zabc + 1024;
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
    const int c = lane % CPB, seg = w * SPW + lane / CPB;
    const int S = (int)(blockDim.x >> 6) * SPW;
    auto C = [&](int q, int s) -> double & { return coef[q * 1024 + s * CPB + c]; };
    const size_t col = (size_t)blockIdx.x * CPB + c;
    const ZSeg sg = zseg(nzp, S, seg);
    ZLane<MMAX, CYC> L;
    zp_load<MMAX, FULL, PAD>(L, data, a, col, sg);
    double out[NQ];
    zp_reduce<MMAX, FULL>(L, a, sg, out);
#pragma unroll
    for (int q = 0; q < NQ; ++q) C(q, seg) = out[q];
    __syncthreads();
    if (w == 0 && lane < CPB) {
        zp_interface<CYC>(
            S, [&](int s, int q) -> double & { return C(q, s); }, [&](int s) -> double & { return C(4, s); },
            [&](int s) -> double & { return C(5, s); }, [&](int s) -> double & { return C(6, s); },
            [&](int s) -> double & { return C(7, s); });
    }
    __syncthreads();
    const double xL = seg > 0 ? C(5, seg - 1) : 0.0;
    const double xR = seg < S - 1 ? C(4, seg + 1) : 0.0;
    if constexpr (CYC) {
        const double xL2 = seg > 0 ? C(7, seg - 1) : 0.0;
        const double xR2 = seg < S - 1 ? C(6, seg + 1) : 0.0;
        zp_finish<MMAX, FULL>(L, a, sg, xL, xR, xL2, xR2);
        // Sherman-Morrison: the column's first and last values of A'^-1 f and
        // A'^-1 u come from its first and last segment
        double y0, z0, yl, zl;
        zp_ends<MMAX, FULL>(L, sg, &y0, &z0, &yl, &zl);
        if (seg == 0) { ends[c] = y0; ends[64 + c] = z0; }
        if (seg == S - 1) { ends[128 + c] = yl; ends[192 + c] = zl; }
        __syncthreads();
        zp_sherman_morrison<MMAX, FULL>(L, a, sg, ends[c], ends[64 + c], ends[128 + c], ends[192 + c]);
    } else {
        zp_finish<MMAX, FULL>(L, a, sg, xL, xR);
    }
    zp_store<MMAX, FULL, PAD>(L, data, a, col, sg);
    if (a.singular && blockIdx.x == 0) {
        // the singular column, left out above: projected rhs, pinned last
        // row, zero weighted mean, by one thread with coef as workspace
        __syncthreads();
        if (threadIdx.x == 0) zsolve_singular_ws<T>(0, data, a, coef, coef + 512, 1);
    }
}

template <typename T>
static int launch_zsolve(const Problem &pb, const Work &w, T *data, double *removed, const int *done, hipStream_t s)
{
    const size_t plane = (size_t)pb.nx * pb.ny;
    const ZPart zp = zpart_shape(pb.nz, pb.cyclic != 0);
    ZArgs za = zargs(pb, w, removed);
    if (zp.mmax == 0) {
        hipLaunchKernelGGL(k_zsolve<T>, dim3((unsigned)((plane + 255) / 256)), dim3(256), 0, s, data, za, done);
        return check_launch();
    }
    const dim3 grid((unsigned)((plane + zp.cpb - 1) / zp.cpb)), block(zp.threads);
    const int S = (zp.threads / 64) * (64 / zp.cpb);
    const bool full = pb.nz == S * zp.mmax;  // every segment holds mmax levels
    // a FULL 16-level kernel keeps both segment sweeps unrolled in registers;
    // with at most 768 threads per block its register limit is 168, not 128
    const bool small = zp.threads <= 768;
#define CANS_ZP(MM, CPB, NT, FULLV, CYCV) \
    hipLaunchKernelGGL((k_zsolve_part<T, MM, CPB, NT, FULLV, CYCV>), grid, block, 0, s, data, za, done)
    if (pb.cyclic) {  // nz <= 128: 8-level segments of 64 columns
        if (full) CANS_ZP(8, 64, 1024, true, true); else CANS_ZP(8, 64, 1024, false, true);
        return check_launch();
    }
#undef CANS_ZP
    // non-periodic z always runs full segments: a ragged nz is padded to
    // S * mmax levels with decoupled rows (the level guards of a ragged
    // split cost ~15 % at nz = 383)
#define CANS_ZP(MM, CPB, NT, PADV) \
    hipLaunchKernelGGL((k_zsolve_part<T, MM, CPB, NT, true, false, PADV>), grid, block, 0, s, data, za, done)
#define CANS_ZP2(MM, CPB, NT) do { if (full) CANS_ZP(MM, CPB, NT, false); else CANS_ZP(MM, CPB, NT, true); } while (0)
    if (zp.mmax == 8) {
        CANS_ZP2(8, 64, 1024);
    } else if (zp.cpb == 64) {
        if (small) CANS_ZP2(16, 64, 768); else CANS_ZP2(16, 64, 1024);
    } else {
        if (small) CANS_ZP2(16, 32, 768); else CANS_ZP2(16, 32, 1024);
    }
#undef CANS_ZP2
#undef CANS_ZP
    return check_launch();
}

static ZArgs zargs(const Problem &pb, const Work &w, double *removed)
{
    ZArgs a;
    a.nx = pb.nx; a.ny = pb.ny; a.nz = pb.nz;
    a.za = pb.d_za; a.zb = pb.d_zb; a.zc = pb.d_zc;
    a.lamx = pb.ax.d_lam; a.lamy = pb.ay.d_lam;
    a.dzf = pb.d_dzf; a.wsum = pb.wsum; a.scale = pb.scale;
    a.cyclic = pb.cyclic; a.singular = pb.singular;
    a.wc = w.wc; a.wd = w.wd; a.wz = w.wz;
    a.removed = removed;
    return a;
}

int launch_zsolve_f64(const Problem &pb, const Work &w, double *data, double *removed, hipStream_t s)
{
    return launch_zsolve<double>(pb, w, data, removed, nullptr, s);
}

int launch_zsolve_32(const Problem &pb, const Work &w, float *data, double *removed, const int *done, hipStream_t s)
{
    return launch_zsolve<float>(pb, w, data, removed, done, s);
}
}  // namespace cans

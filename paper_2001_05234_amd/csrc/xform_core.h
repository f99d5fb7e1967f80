// xform_core.h -- real-to-real transforms of Section 2 ("FFT-based Poisson
// solver") built on one complex FFT of half length, evaluated on a tile of L
// lines held in LDS.
//
// Every transform is a phase sequence over two LDS buffers (b0, b1) of n*L
// reals each, element (index e, line l) at [e*L + l]:
//   load   global -> b1 (real line data)                 (kernel specific)
//   pre    b1 -> b0: pack the n reals of a line into M = n/2 complex values,
//          with the reorder / sign / twiddle the boundary pair needs
//   stage  Stockham radix-r pass (decimation in frequency), ping-pong b0/b1
//   post   final -> other buffer: unpack M complex values into n reals
//   store  other buffer -> global                         (kernel specific)
// Phases only read what earlier phases wrote, so a barrier between phases is
// the only synchronisation; the same functions run on the host in the tests.
//
// Transforms (n even, M = n/2, unnormalised, rows indexed by q):
//   P  forward: real DFT, layout [X_0, X_M, Re X_1, Im X_1, ..., Re X_{M-1},
//      Im X_{M-1}], X_l = sum x_i e^{-2 pi i l i/n};  inverse: the matching
//      half-complex synthesis, x = X_0 + (-1)^i X_M + 2 sum Re(X_l e^{+...}).
//   NN forward DCT-II (Makhoul's even/odd reorder + real DFT + quarter-wave
//      twiddle); inverse DCT-III (X_0 + 2 sum ...).
//   DD forward DST-II = reversed DCT-II of (-1)^i x; inverse DST-III.
//   ND DCT-IV through an M-point complex FFT with pre/post twiddles; its own
//      inverse up to n/2.
//   DN DST-IV = (-1)^q DCT-IV of the reversed line; own inverse up to n/2.
// With B the inverse listed, B T = s I with s = n (P, NN, DD) or n/2 (ND, DN).
#pragma once

#include <hip/hip_runtime.h>

#define CANS_HD __host__ __device__ inline

namespace cans {

enum Kind { K_P = 0, K_NN = 1, K_DD = 2, K_ND = 3, K_DN = 4 };

constexpr int kMaxStages = 24;

template <typename T>
struct cx {
    T re, im;
};

template <typename T> CANS_HD cx<T> mk(T r, T i) { cx<T> c; c.re = r; c.im = i; return c; }
template <typename T> CANS_HD cx<T> operator+(cx<T> a, cx<T> b) { return mk(a.re + b.re, a.im + b.im); }
template <typename T> CANS_HD cx<T> operator-(cx<T> a, cx<T> b) { return mk(a.re - b.re, a.im - b.im); }
template <typename T> CANS_HD cx<T> operator*(cx<T> a, cx<T> b)
{
    return mk(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
template <typename T> CANS_HD cx<T> scal(cx<T> a, T s) { return mk(a.re * s, a.im * s); }
template <typename T> CANS_HD cx<T> conj(cx<T> a) { return mk(a.re, -a.im); }
// multiply by +i or -i
template <typename T> CANS_HD cx<T> mul_pi(cx<T> a) { return mk(-a.im, a.re); }
template <typename T> CANS_HD cx<T> mul_ni(cx<T> a) { return mk(a.im, -a.re); }
// multiply by -i (forward) or +i (inverse): the quarter turn of a DFT
template <bool FWD, typename T> CANS_HD cx<T> qturn(cx<T> a) { return FWD ? mul_ni(a) : mul_pi(a); }
// a * w (forward) or a * conj(w) (inverse)
template <bool FWD, typename T> CANS_HD cx<T> twid(cx<T> a, cx<T> w) { return FWD ? a * w : a * conj(w); }

// ---------------------------------------------------------------------------
// small DFTs, A_u = sum_j a_j w^{j u}, w = e^{-2 pi i/r} (forward) or e^{+} (inverse)
template <bool FWD, typename T>
CANS_HD void dft2(cx<T> *a)
{
    cx<T> t = a[0] - a[1];
    a[0] = a[0] + a[1];
    a[1] = t;
}

template <bool FWD, typename T>
CANS_HD void dft3(cx<T> *a)
{
    const T h = T(0.866025403784438646763723170752936183);  // sqrt(3)/2
    cx<T> t = a[1] + a[2];
    cx<T> s = qturn<FWD>(scal(a[1] - a[2], h));
    cx<T> m = a[0] - scal(t, T(0.5));
    a[0] = a[0] + t;
    a[1] = m + s;
    a[2] = m - s;
}

template <bool FWD, typename T>
CANS_HD void dft4(cx<T> *a)
{
    cx<T> s02 = a[0] + a[2], d02 = a[0] - a[2];
    cx<T> s13 = a[1] + a[3], d13 = qturn<FWD>(a[1] - a[3]);
    a[0] = s02 + s13;
    a[2] = s02 - s13;
    a[1] = d02 + d13;
    a[3] = d02 - d13;
}

template <bool FWD, typename T>
CANS_HD void dft5(cx<T> *a)
{
    const T c1 = T(0.309016994374947424102293417182819059);   // cos(2pi/5)
    const T c2 = T(-0.809016994374947424102293417182819059);  // cos(4pi/5)
    const T s1 = T(0.951056516295153572116439333379382143);   // sin(2pi/5)
    const T s2 = T(0.587785252292473129168705954639072769);   // sin(4pi/5)
    cx<T> t1 = a[1] + a[4], t2 = a[2] + a[3], t3 = a[1] - a[4], t4 = a[2] - a[3];
    cx<T> b1 = a[0] + scal(t1, c1) + scal(t2, c2);
    cx<T> b2 = a[0] + scal(t1, c2) + scal(t2, c1);
    cx<T> e1 = qturn<FWD>(scal(t3, s1) + scal(t4, s2));
    cx<T> e2 = qturn<FWD>(scal(t3, s2) - scal(t4, s1));
    a[0] = a[0] + t1 + t2;
    a[1] = b1 + e1;
    a[4] = b1 - e1;
    a[2] = b2 + e2;
    a[3] = b2 - e2;
}

template <bool FWD, typename T>
CANS_HD void dft8(cx<T> *a)
{
    const T r = T(0.707106781186547524400844362104849039);
    cx<T> e[4] = {a[0], a[2], a[4], a[6]}, o[4] = {a[1], a[3], a[5], a[7]};
    dft4<FWD>(e);
    dft4<FWD>(o);
    // o_u *= w8^u
    o[1] = FWD ? mk(r * (o[1].re + o[1].im), r * (o[1].im - o[1].re))
               : mk(r * (o[1].re - o[1].im), r * (o[1].im + o[1].re));
    o[2] = qturn<FWD>(o[2]);
    o[3] = FWD ? mk(r * (o[3].im - o[3].re), -r * (o[3].re + o[3].im))
               : mk(-r * (o[3].re + o[3].im), r * (o[3].re - o[3].im));
    for (int u = 0; u < 4; ++u) {
        a[u] = e[u] + o[u];
        a[u + 4] = e[u] - o[u];
    }
}

template <bool FWD, typename T>
CANS_HD void dft_r(const int r, cx<T> *a)
{
    switch (r) {
    case 2: dft2<FWD>(a); break;
    case 3: dft3<FWD>(a); break;
    case 4: dft4<FWD>(a); break;
    case 5: dft5<FWD>(a); break;
    default: dft8<FWD>(a); break;
    }
}

// ---------------------------------------------------------------------------
// Geometry of one transform tile.
struct XGeom {
    int n;      // real length (even)
    int M;      // n / 2
    int L;      // lines per tile (power of two)
    int lgL;
    int nst;    // FFT stages
    int rad[kMaxStages];
    int str[kMaxStages];  // s of each stage (product of earlier radices)
};

// Twiddle table of one axis (complex, in the compute type), offsets in units
// of cx<T>:
//   [0, M)          W_M^j = e^{-2 pi i j/M}              FFT stages
//   [M, 2M)         W_n^k = e^{-2 pi i k/n}              real-DFT split
//   [2M, 3M+1)      (cos(pi q/2n), sin(pi q/2n))         DCT-II quarter wave
//   [3M+1, 4M+1)    e^{-i pi (4m+1)/(4n)}                 DCT-IV pre
//   [4M+1, 5M+1)    e^{-i pi k/n}                         DCT-IV post
CANS_HD int tw_fft(int) { return 0; }
CANS_HD int tw_split(int M) { return M; }
CANS_HD int tw_qw(int M) { return 2 * M; }
CANS_HD int tw_pre4(int M) { return 3 * M + 1; }
CANS_HD int tw_post4(int M) { return 4 * M + 1; }
CANS_HD int tw_size(int M) { return 5 * M + 1; }

// real element e of line l in a tile buffer
template <typename T> CANS_HD T &R(T *b, const XGeom &g, int e, int l) { return b[e * g.L + l]; }
template <typename T> CANS_HD cx<T> &C(T *b, const XGeom &g, int m, int l)
{
    return reinterpret_cast<cx<T> *>(b)[m * g.L + l];
}

// Makhoul's even/odd reorder: v_j = x_{2j} (j < M), x_{2(n-1-j)+1} (j >= M);
// returns the source index and whether it is odd.
CANS_HD int mk_src(int j, int n, int M) { return j < M ? 2 * j : 2 * (n - 1 - j) + 1; }

// ---- pre: b1 (real) -> b0 (complex) --------------------------------------
template <int KIND, bool FWD, typename T>
CANS_HD void phase_pre(int tid, int nt, const XGeom &g, T *b0, const T *b1c, const cx<T> *tw)
{
    T *b1 = const_cast<T *>(b1c);
    const int n = g.n, M = g.M;
    for (int w = tid; w < M * g.L; w += nt) {
        const int m = w >> g.lgL, l = w & (g.L - 1);
        cx<T> z;
        if (KIND == K_ND || KIND == K_DN) {
            T a = R(b1, g, 2 * m, l), b = R(b1, g, n - 1 - 2 * m, l);
            z = (KIND == K_ND) ? mk(a, b) : mk(b, a);
            z = z * tw[tw_pre4(M) + m];
        } else if (FWD) {
            if (KIND == K_P) {
                z = mk(R(b1, g, 2 * m, l), R(b1, g, 2 * m + 1, l));
            } else {
                int s0 = mk_src(2 * m, n, M), s1 = mk_src(2 * m + 1, n, M);
                T v0 = R(b1, g, s0, l), v1 = R(b1, g, s1, l);
                if (KIND == K_DD) {  // (-1)^i on the input
                    if (s0 & 1) v0 = -v0;
                    if (s1 & 1) v1 = -v1;
                }
                z = mk(v0, v1);
            }
        } else {
            // inverse: build the half spectrum X_k, X_{M-k} of a real line,
            // then Z_k = (X_k + conj X_{M-k}) + i (X_k - conj X_{M-k}) W_n^{-k}
            cx<T> Xk, Xc;
            const int kc = M - m;  // in 1..M
            if (KIND == K_P) {
                Xk = (m == 0) ? mk(R(b1, g, 0, l), T(0)) : mk(R(b1, g, 2 * m, l), R(b1, g, 2 * m + 1, l));
                Xc = (kc == M) ? mk(R(b1, g, 1, l), T(0)) : mk(R(b1, g, 2 * kc, l), R(b1, g, 2 * kc + 1, l));
            } else {
                // V_q = e^{i pi q/2n} (Y_q - i Y_{n-q}); V_0 = Y_0; V_M = sqrt2 Y_M.
                // DD reads its input reversed: Y'_q = Y_{n-1-q}.
                auto Y = [&](int q) -> T { return R(b1, g, KIND == K_DD ? n - 1 - q : q, l); };
                auto V = [&](int q) -> cx<T> {
                    if (q == 0) return mk(Y(0), T(0));
                    if (q == M) return mk(T(1.41421356237309504880168872420969808) * Y(M), T(0));
                    cx<T> cs = tw[tw_qw(M) + q];
                    return cs * mk(Y(q), -Y(n - q));
                };
                Xk = V(m);
                Xc = V(kc);
            }
            Xc = conj(Xc);
            cx<T> E = Xk + Xc;
            cx<T> O = (Xk - Xc) * conj(tw[tw_split(M) + m]);
            z = E + mul_pi(O);
        }
        C(b0, g, m, l) = z;
    }
}

// ---- one Stockham stage: src -> dst ---------------------------------------
// Butterfly (q, p) of a stage with radix RAD and stride s reads
// x[q + s (p + j m)], j < RAD, m = M/(s RAD), and writes
// y[q + s (RAD p + u)] = DFT_RAD(x)_u * W_M^{p u s}.
template <int RAD, bool FWD, typename T>
CANS_HD void stage_rad(int tid, int nt, const XGeom &g, int s, T *src, T *dst, const cx<T> *tw)
{
    const int M = g.M;
    const int m = M / (s * RAD);
    const int nb = (M / RAD) << g.lgL;
    for (int w = tid; w < nb; w += nt) {
        const int l = w & (g.L - 1), b = w >> g.lgL;
        const int q = b % s, p = b / s;
        cx<T> a[RAD];
#pragma unroll
        for (int j = 0; j < RAD; ++j) a[j] = C(src, g, q + s * (p + j * m), l);
        dft_r<FWD>(RAD, a);
        C(dst, g, q + s * (RAD * p), l) = a[0];
#pragma unroll
        for (int u = 1; u < RAD; ++u)
            C(dst, g, q + s * (RAD * p + u), l) = twid<FWD>(a[u], tw[tw_fft(M) + p * u * s]);
    }
}

template <bool FWD, typename T>
CANS_HD void phase_stage(int tid, int nt, const XGeom &g, int st, const T *srcc, T *dst, const cx<T> *tw)
{
    T *src = const_cast<T *>(srcc);
    const int s = g.str[st];
    switch (g.rad[st]) {
    case 2: stage_rad<2, FWD>(tid, nt, g, s, src, dst, tw); break;
    case 3: stage_rad<3, FWD>(tid, nt, g, s, src, dst, tw); break;
    case 4: stage_rad<4, FWD>(tid, nt, g, s, src, dst, tw); break;
    case 5: stage_rad<5, FWD>(tid, nt, g, s, src, dst, tw); break;
    default: stage_rad<8, FWD>(tid, nt, g, s, src, dst, tw); break;
    }
}

// ---- post: final complex buffer -> real buffer ----------------------------
template <int KIND, bool FWD, typename T>
CANS_HD void phase_post(int tid, int nt, const XGeom &g, const T *srcc, T *out, const cx<T> *tw)
{
    T *src = const_cast<T *>(srcc);
    const int n = g.n, M = g.M;
    for (int w = tid; w < M * g.L; w += nt) {
        const int k = w >> g.lgL, l = w & (g.L - 1);
        cx<T> Z = C(src, g, k, l);
        if (KIND == K_ND || KIND == K_DN) {
            cx<T> u = Z * tw[tw_post4(M) + k];
            R(out, g, 2 * k, l) = u.re;
            R(out, g, n - 1 - 2 * k, l) = (KIND == K_ND) ? -u.im : u.im;
        } else if (FWD) {
            // split the M-point FFT of the packed line into the real DFT V_k
            cx<T> V;
            if (k == 0) {
                V = mk(Z.re + Z.im, T(0));
            } else {
                cx<T> Zc = conj(C(src, g, M - k, l));
                cx<T> E = scal(Z + Zc, T(0.5));
                cx<T> O = scal(mul_ni(Z - Zc), T(0.5));
                V = E + tw[tw_split(M) + k] * O;
            }
            if (KIND == K_P) {
                if (k == 0) {
                    R(out, g, 0, l) = V.re;
                    R(out, g, 1, l) = Z.re - Z.im;
                } else {
                    R(out, g, 2 * k, l) = V.re;
                    R(out, g, 2 * k + 1, l) = V.im;
                }
            } else {
                // DCT-II: X_q = c Re V_q + s Im V_q, X_{n-q} = s Re V_q - c Im V_q;
                // DST-II stores X_q at n-1-q
                auto put = [&](int q, T v) { R(out, g, KIND == K_DD ? n - 1 - q : q, l) = v; };
                if (k == 0) {
                    put(0, V.re);
                    put(M, (Z.re - Z.im) * tw[tw_qw(M) + M].re);
                } else {
                    cx<T> cs = tw[tw_qw(M) + k];
                    put(k, cs.re * V.re + cs.im * V.im);
                    put(n - k, cs.im * V.re - cs.re * V.im);
                }
            }
        } else {
            if (KIND == K_P) {
                R(out, g, 2 * k, l) = Z.re;
                R(out, g, 2 * k + 1, l) = Z.im;
            } else {
                // undo Makhoul's reorder; DST-III multiplies by (-1)^i
                int d0 = mk_src(2 * k, n, M), d1 = mk_src(2 * k + 1, n, M);
                T v0 = Z.re, v1 = Z.im;
                if (KIND == K_DD) {
                    if (d0 & 1) v0 = -v0;
                    if (d1 & 1) v1 = -v1;
                }
                R(out, g, d0, l) = v0;
                R(out, g, d1, l) = v1;
            }
        }
    }
}

// Run pre, stages and post on a tile whose real data sits in b1; the result
// (real) ends in the returned buffer.  `sync` is the barrier between phases.
// Run with tid = 0, nt = 1 and an empty `sync`, it is the serial reference
// execution of the same arithmetic (used by the host-side tests).
template <int KIND, bool FWD, typename T, typename Sync>
CANS_HD T *tile_transform(int tid, int nt, const XGeom &g, T *b0, T *b1, const cx<T> *tw, Sync sync)
{
    // DCT-IV and DST-IV are their own inverses: the FFT runs forward both ways
    constexpr bool FFTF = FWD || KIND == K_ND || KIND == K_DN;
    phase_pre<KIND, FWD>(tid, nt, g, b0, b1, tw);
    sync();
    T *src = b0, *dst = b1;
    for (int st = 0; st < g.nst; ++st) {
        phase_stage<FFTF>(tid, nt, g, st, src, dst, tw);
        sync();
        T *t = src; src = dst; dst = t;
    }
    phase_post<KIND, FWD>(tid, nt, g, src, dst, tw);
    sync();
    return dst;
}

}  // namespace cans

// xform_core.h -- real-to-real transforms of Section 2 ("FFT-based Poisson
// solver") built on one complex FFT of half length, evaluated on a tile of L
// lines held in LDS.
//
// A transform of a tile is:
//   stage 0  each butterfly reads its inputs straight from global memory
//            through the boundary pair's packing map (n reals of a line ->
//            M = n/2 complex values, with reorder / sign / pre-twiddle) and
//            writes its outputs to the LDS tile;
//   stage t  Stockham radix-r pass (decimation in frequency) in place in LDS:
//            inputs to registers, barrier, outputs to LDS, barrier;
//   post     each output pair reads Z_k and Z_{M-k} from LDS, applies the
//            unpacking map and writes the reals straight to global memory.
// Loads and stores go through functors, so the same functions run the
// kernels (block threads, barriers) and the serial host build of the tests
// (one thread, out of place).
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
//
// Fields located on the faces of an axis (nl unknowns per line, n = 2M the
// length of the extended line the FFT sees):
//   S1  DST-I of nl = M-1 values, X_q = 2 sum_i x_i sin(pi (q+1)(i+1)/M):
//       the real DFT of the line extended odd about 0 and M (zero there) to
//       2M reals is -i X; its own inverse up to s = 2M.
//   C1  DCT-I of nl = M+1 values, X_q = x_0 + (-1)^q x_M + 2 sum_{0<i<M}
//       x_i cos(pi q i/M): the real DFT of the line extended even about 0
//       and M; its own inverse up to s = 2M.
//   FDN, FND  (Dirichlet face, Neumann face) and (Neumann face, Dirichlet
//       face): the type-III sine and cosine transforms, i.e. the DD and NN
//       pairs above run the other way round (DST-III forward, DST-II back;
//       DCT-III forward, DCT-II back), s = n = nl.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#define CANS_HD __host__ __device__ inline __attribute__((always_inline))

namespace cans {

enum Kind { K_P = 0, K_NN = 1, K_DD = 2, K_ND = 3, K_DN = 4, K_S1 = 5, K_C1 = 6, K_FDN = 7, K_FND = 8 };

// the transform a kind runs (FDN and FND run DD and NN backwards), whether
// it runs it backwards, and whether it is its own inverse
constexpr int base_kind(int k) { return k == K_FDN ? K_DD : (k == K_FND ? K_NN : k); }
constexpr bool flipped(int k) { return k == K_FDN || k == K_FND; }
constexpr bool own_inverse(int k) { return k == K_ND || k == K_DN || k == K_S1 || k == K_C1; }
// the packing map of the transform reads each input real twice (synthesis
// of a half spectrum, or an extended line)
constexpr bool reads_twice(int k, bool fwd)
{
    return base_kind(k) == K_S1 || base_kind(k) == K_C1 ||
           ((flipped(k) ? fwd : !fwd) && (base_kind(k) == K_P || base_kind(k) == K_NN || base_kind(k) == K_DD));
}
// length of the extended real line of a kind with nl unknowns a line
CANS_HD int fft_len(int kind, int nl) { return kind == K_S1 ? 2 * (nl + 1) : (kind == K_C1 ? 2 * (nl - 1) : nl); }

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
// Exact division of n < 2^16 by a runtime d < 2^16: q = hi32(n * mag).
CANS_HD unsigned mag_of(unsigned d) { return d <= 1 ? 0u : (unsigned)((1ull << 32) / d + 1); }
CANS_HD unsigned udiv(unsigned n, unsigned d, unsigned mag)
{
    if (d <= 1) return n;
#if defined(__HIP_DEVICE_COMPILE__)
    return __umulhi(n, mag);
#else
    return (unsigned)(((unsigned long long)n * mag) >> 32);
#endif
}

// Geometry of one transform tile.
struct XGeom {
    int n;      // real length of the (extended) line the FFT sees (even)
    int nl;     // reals of a line in memory: n, or n/2 -+ 1 for S1 / C1
    int M;      // n / 2
    int L;      // lines per tile (power of two)
    int lgL;
    int RS;     // row stride of an x tile in complex slots (with padding)
    int psh;    // x tiles: one pad slot every 2^psh slots (256-byte LDS rows)
    int nst;    // FFT stages
    unsigned magM;
    unsigned magN;     // magic for / nl
    int rad[kMaxStages];
    int str[kMaxStages];       // s of each stage (product of earlier radices)
    unsigned mag_s[kMaxStages];   // magic for / s
    unsigned mag_nb[kMaxStages];  // magic for / (M / rad)
};

enum { AX_X = 0, AX_Y = 1 };

// LDS tile of L lines of M complex values.
//   x tiles: line-major, slot (m, l) at l*RS + m + (m >> psh);
//   y tiles: element-major, slot (m, l) at m*(L+1) + l.
template <int AXIS, typename T>
struct Tile {
    cx<T> *c;
    int L, RS, psh;
    CANS_HD cx<T> &at(int m, int l) const
    {
        return AXIS == AX_X ? c[l * RS + m + (m >> psh)] : c[m * (L + 1) + l];
    }
};

// complex slots a tile needs
CANS_HD int tile_slots(int axis, const XGeom &g) { return axis == AX_X ? g.L * g.RS : g.M * (g.L + 1); }

// work item w of `per` items per line -> (line, item)
template <int AXIS>
CANS_HD void split_item(int w, int per, unsigned mag, int lgL, int L, int &l, int &it)
{
    if (AXIS == AX_X) {
        l = (int)udiv((unsigned)w, (unsigned)per, mag);
        it = w - l * per;
    } else {
        l = w & (L - 1);
        it = w >> lgL;
    }
}

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

// Makhoul's even/odd reorder: v_j = x_{2j} (j < M), x_{2(n-1-j)+1} (j >= M).
CANS_HD int mk_src(int j, int n, int M) { return j < M ? 2 * j : 2 * (n - 1 - j) + 1; }

// ---- packing map: z_m of line l from the line's reals src(e) ---------------
template <int KIND, bool FWD, typename T, typename Src>
CANS_HD cx<T> pack(int m, const XGeom &g, const Src &src, const cx<T> *tw)
{
    const int n = g.n, M = g.M;
    if (KIND == K_S1 || KIND == K_C1) {
        // the line extended to 2M reals: odd about 0 and M (zero there) for
        // DST-I, even about them for DCT-I
        auto ext = [&](int j) -> T {
            if (KIND == K_S1) {
                if (j == 0 || j == M) return T(0);
                return j < M ? src(j - 1) : -src(2 * M - 1 - j);
            }
            return src(j <= M ? j : 2 * M - j);
        };
        return mk(ext(2 * m), ext(2 * m + 1));
    }
    if (KIND == K_ND || KIND == K_DN) {
        const T a = src(2 * m), b = src(n - 1 - 2 * m);
        return ((KIND == K_ND) ? mk(a, b) : mk(b, a)) * tw[tw_pre4(M) + m];
    }
    if (FWD) {
        if (KIND == K_P) return mk(src(2 * m), src(2 * m + 1));
        const int s0 = mk_src(2 * m, n, M), s1 = mk_src(2 * m + 1, n, M);
        T v0 = src(s0), v1 = src(s1);
        if (KIND == K_DD) {  // (-1)^i on the input
            if (s0 & 1) v0 = -v0;
            if (s1 & 1) v1 = -v1;
        }
        return mk(v0, v1);
    }
    // inverse: half spectrum X_k, X_{M-k} of a real line, then
    // Z_k = (X_k + conj X_{M-k}) + i (X_k - conj X_{M-k}) W_n^{-k}
    cx<T> Xk, Xc;
    const int kc = M - m;  // in 1..M
    if (KIND == K_P) {
        Xk = (m == 0) ? mk(src(0), T(0)) : mk(src(2 * m), src(2 * m + 1));
        Xc = (kc == M) ? mk(src(1), T(0)) : mk(src(2 * kc), src(2 * kc + 1));
    } else {
        // V_q = e^{i pi q/2n} (Y_q - i Y_{n-q}); V_0 = Y_0; V_M = sqrt2 Y_M;
        // DST-III reads its input reversed: Y'_q = Y_{n-1-q}
        auto Y = [&](int q) -> T { return src(KIND == K_DD ? n - 1 - q : q); };
        auto V = [&](int q) -> cx<T> {
            if (q == 0) return mk(Y(0), T(0));
            if (q == M) return mk(T(1.41421356237309504880168872420969808) * Y(M), T(0));
            return tw[tw_qw(M) + q] * mk(Y(q), -Y(n - q));
        };
        Xk = V(m);
        Xc = V(kc);
    }
    Xc = conj(Xc);
    const cx<T> E = Xk + Xc;
    const cx<T> O = (Xk - Xc) * conj(tw[tw_split(M) + m]);
    return E + mul_pi(O);
}

// ---- unpacking map: the reals of output pair k from Z (the FFT result) -----
// put(q, v) receives output real q of the line.
// put2(q, a, b) receives the adjacent reals q, q+1 (the periodic pair's
// outputs), put(q, v) every other one.
template <int KIND, bool FWD, typename T, typename ZAt, typename Put, typename Put2>
CANS_HD void unpack(int k, const XGeom &g, const ZAt &Z, const Put &put, const Put2 &put2, const cx<T> *tw)
{
    const int n = g.n, M = g.M;
    const cx<T> z = Z(k);
    if (KIND == K_S1 || KIND == K_C1) {
        // V_k of the extended line (the real-DFT split below); DST-I keeps
        // -Im V_k, k = 1..M-1, DCT-I Re V_k, k = 0..M
        if (k == 0) {
            if (KIND == K_C1) {
                put(0, z.re + z.im);
                put(M, z.re - z.im);
            }
            return;
        }
        const cx<T> zc = conj(Z(M - k));
        const cx<T> E = scal(z + zc, T(0.5));
        const cx<T> O = scal(mul_ni(z - zc), T(0.5));
        const cx<T> V = E + tw[tw_split(M) + k] * O;
        if (KIND == K_S1) put(k - 1, -V.im);
        else put(k, V.re);
        return;
    }
    if (KIND == K_ND || KIND == K_DN) {
        const cx<T> u = z * tw[tw_post4(M) + k];
        put(2 * k, u.re);
        put(n - 1 - 2 * k, (KIND == K_ND) ? -u.im : u.im);
        return;
    }
    if (FWD) {
        // split the M-point FFT of the packed line into the real DFT V_k
        cx<T> V;
        if (k == 0) {
            V = mk(z.re + z.im, T(0));
        } else {
            const cx<T> zc = conj(Z(M - k));
            const cx<T> E = scal(z + zc, T(0.5));
            const cx<T> O = scal(mul_ni(z - zc), T(0.5));
            V = E + tw[tw_split(M) + k] * O;
        }
        if (KIND == K_P) {
            if (k == 0) {
                put2(0, V.re, z.re - z.im);
            } else {
                put2(2 * k, V.re, V.im);
            }
            return;
        }
        // DCT-II: X_q = c Re V_q + s Im V_q, X_{n-q} = s Re V_q - c Im V_q;
        // DST-II stores X_q at n-1-q
        auto out = [&](int q, T v) { put(KIND == K_DD ? n - 1 - q : q, v); };
        if (k == 0) {
            out(0, V.re);
            out(M, (z.re - z.im) * tw[tw_qw(M) + M].re);
        } else {
            const cx<T> cs = tw[tw_qw(M) + k];
            out(k, cs.re * V.re + cs.im * V.im);
            out(n - k, cs.im * V.re - cs.re * V.im);
        }
        return;
    }
    if (KIND == K_P) {
        put2(2 * k, z.re, z.im);
        return;
    }
    // undo Makhoul's reorder; DST-III multiplies by (-1)^i
    const int d0 = mk_src(2 * k, n, M), d1 = mk_src(2 * k + 1, n, M);
    T v0 = z.re, v1 = z.im;
    if (KIND == K_DD) {
        if (d0 & 1) v0 = -v0;
        if (d1 & 1) v1 = -v1;
    }
    put(d0, v0);
    put(d1, v1);
}

// ---- one Stockham stage ----------------------------------------------------
// Butterfly (q, p) of a stage with radix RAD and stride s reads
// x[q + s (p + j m)], j < RAD, m = M/(s RAD), and writes
// y[q + s (RAD p + u)] = DFT_RAD(x)_u * W_M^{p u s}.  The twiddle W^{p s}
// is read once; its powers are formed by at most three products.
template <int RAD, bool FWD, typename T>
CANS_HD void twiddle_powers(cx<T> w1, cx<T> *w)
{
    w[1] = w1;
    if (RAD > 2) w[2] = w1 * w1;
    if (RAD > 3) w[3] = w[2] * w1;
    if (RAD > 4) w[4] = w[2] * w[2];
    if (RAD > 5) { w[5] = w[4] * w1; w[6] = w[4] * w[2]; w[7] = w[4] * w[3]; }
}

// capacity of the in-place stage: complex values a thread holds
constexpr int kMaxC = 16;

// IN(m, l) gives the stage input (LDS, or the packing map for stage 0).
// INPLACE: the inputs of all of this thread's butterflies are read before
// `sync` and the outputs written after it, so src and dst may be one tile.
template <int RAD, bool FWD, int AXIS, bool INPLACE, typename T, typename In, typename Sync>
CANS_HD void stage_rad(int tid, int nt, const XGeom &g, int st, const In &in, const Tile<AXIS, T> &dst,
                       const cx<T> *tw, const Sync &sync)
{
    const int M = g.M;
    const int s = g.str[st];
    const int m = M / (s * RAD);
    const int per = M / RAD;
    const int nb = per * g.L;
    auto butterfly_io = [&](int w, int &l, int &q, int &p) {
        int b;
        split_item<AXIS>(w, per, g.mag_nb[st], g.lgL, g.L, l, b);
        p = (int)udiv((unsigned)b, (unsigned)s, g.mag_s[st]);
        q = b - p * s;
    };
    auto finish = [&](int l, int q, int p, cx<T> *a) {
        dft_r<FWD>(RAD, a);
        cx<T> wp[8];
        twiddle_powers<RAD, FWD>(tw[tw_fft(M) + p * s], wp);
        dst.at(q + s * (RAD * p), l) = a[0];
#pragma unroll
        for (int u = 1; u < RAD; ++u) dst.at(q + s * (RAD * p + u), l) = twid<FWD>(a[u], wp[u]);
    };
    if (INPLACE) {
        constexpr int NB = kMaxC / RAD;
        cx<T> a[NB][RAD];
#pragma unroll
        for (int jb = 0; jb < NB; ++jb) {
            const int w = tid + jb * nt;
            if (w < nb) {
                int l, q, p;
                butterfly_io(w, l, q, p);
#pragma unroll
                for (int j = 0; j < RAD; ++j) a[jb][j] = in(q + s * (p + j * m), l);
            }
        }
        sync();
#pragma unroll
        for (int jb = 0; jb < NB; ++jb) {
            const int w = tid + jb * nt;
            if (w < nb) {
                int l, q, p;
                butterfly_io(w, l, q, p);
                finish(l, q, p, a[jb]);
            }
        }
    } else {
        for (int w = tid; w < nb; w += nt) {
            int l, q, p;
            butterfly_io(w, l, q, p);
            cx<T> a[RAD];
#pragma unroll
            for (int j = 0; j < RAD; ++j) a[j] = in(q + s * (p + j * m), l);
            finish(l, q, p, a);
        }
    }
    sync();
}

template <bool FWD, int AXIS, bool INPLACE, typename T, typename In, typename Sync>
CANS_HD void stage_any(int tid, int nt, const XGeom &g, int st, const In &in, const Tile<AXIS, T> &dst,
                       const cx<T> *tw, const Sync &sync)
{
    switch (g.rad[st]) {
    case 2: stage_rad<2, FWD, AXIS, INPLACE>(tid, nt, g, st, in, dst, tw, sync); break;
    case 3: stage_rad<3, FWD, AXIS, INPLACE>(tid, nt, g, st, in, dst, tw, sync); break;
    case 4: stage_rad<4, FWD, AXIS, INPLACE>(tid, nt, g, st, in, dst, tw, sync); break;
    case 5: stage_rad<5, FWD, AXIS, INPLACE>(tid, nt, g, st, in, dst, tw, sync); break;
    default: stage_rad<8, FWD, AXIS, INPLACE>(tid, nt, g, st, in, dst, tw, sync); break;
    }
}

// The whole transform of a tile.
//   src(e, l):   real e of input line l (global memory, a computed value, or
//                with SRCTILE the tile itself, filled by the caller)
//   put(q, l, v): real q of output line l
//   ta, tb:      tiles; the kernels pass one tile twice (INPLACE), the host
//                build passes two (ping-pong).
// The caller synchronises before reusing the tile.
template <int KIND, bool FWD, int AXIS, bool INPLACE, bool SRCTILE, typename T, typename Src, typename Put,
          typename Sync>
CANS_HD void tile_transform(int tid, int nt, const XGeom &g, const Src &src, const Put &put, Tile<AXIS, T> ta,
                            Tile<AXIS, T> tb, const cx<T> *tw, const Sync &sync)
{
    // the face pairs FDN / FND run DD / NN backwards; the transforms that
    // are their own inverses run the FFT forward both ways
    constexpr int BK = base_kind(KIND);
    constexpr bool BF = flipped(KIND) ? !FWD : FWD;
    constexpr bool FFTF = BF || own_inverse(BK);
    auto packed = [&](int m, int l) -> cx<T> {
        return pack<BK, BF, T>(m, g, [&](int e) -> T { return src(e, l); }, tw);
    };
    Tile<AXIS, T> cur = ta, nxt = tb;
    if (g.nst == 0) {
        // M = 1: the packed value is the spectrum; each line's slot is read
        // and written by the same thread
        for (int w = tid; w < g.L; w += nt) {
            const cx<T> z = packed(0, w);
            nxt.at(0, w) = z;
        }
        sync();
        cur = nxt;
    } else if (SRCTILE) {
        stage_any<FFTF, AXIS, INPLACE>(tid, nt, g, 0, packed, nxt, tw, sync);
        Tile<AXIS, T> t = cur; cur = nxt; nxt = t;
    } else {
        stage_any<FFTF, AXIS, false>(tid, nt, g, 0, packed, cur, tw, sync);
    }
    for (int st = 1; st < g.nst; ++st) {
        auto lds = [&](int m, int l) -> cx<T> { return cur.at(m, l); };
        stage_any<FFTF, AXIS, INPLACE>(tid, nt, g, st, lds, nxt, tw, sync);
        Tile<AXIS, T> t = cur; cur = nxt; nxt = t;
    }
    const int total = g.M * g.L;
    for (int w = tid; w < total; w += nt) {
        int l, k;
        split_item<AXIS>(w, g.M, g.magM, g.lgL, g.L, l, k);
        // a put that takes two adjacent reals stores them at once
        auto put2 = [&](int q, T v0, T v1) {
            if constexpr (std::is_invocable_v<const Put &, int, int, T, T>) {
                put(q, l, v0, v1);
            } else {
                put(q, l, v0);
                put(q + 1, l, v1);
            }
        };
        unpack<BK, BF, T>(
            k, g, [&](int kk) -> cx<T> { return cur.at(kk, l); }, [&](int q, T v) { put(q, l, v); }, put2, tw);
    }
}

// real e of line l of a tile (the real view used by SRCTILE loads)
template <int AXIS, typename T>
CANS_HD T &tile_real(const Tile<AXIS, T> &t, int e, int l)
{
    return reinterpret_cast<T *>(&t.at(e >> 1, l))[e & 1];
}

}  // namespace cans

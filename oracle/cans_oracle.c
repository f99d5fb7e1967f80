/*
 * cans_oracle.c -- plain, slow, obviously-correct CPU oracle for the direct
 * Poisson solver of Costa, Phillips, Brandt & Fatica, "GPU acceleration of
 * CaNS" (arXiv 2001.05234).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or
 * calls this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, table or constant
 * generator with the GPU library.
 *
 * What it computes (Section 2, "FFT-based Poisson solver"):
 *   - the 7-point second-order discretisation of the Poisson equation on a
 *     staggered grid, eq. (poi), with the z part written in conservative
 *     (flux) form so that a non-uniform z spacing is allowed (the remark
 *     following eq. (poi_reduced); the inverse spacings dzci/dzfi of
 *     Listing 1);
 *   - its solution by eigenfunction expansion: a discrete transform F^x along
 *     x, then F^y along y, which leaves one tridiagonal system in z per
 *     (i,j) wavenumber pair, eq. (poi_reduced), solved by Gauss elimination
 *     without pivoting; then the inverse transforms.
 *
 * The transforms are the plain O(N^2) matrix products with the closed-form
 * eigenvector rows of each boundary-condition pair; the paper leaves those
 * formulas to its references (Schumann & Sweet 1988), so the rows and the
 * eigenvalues mu(q) used here are derived from the ghost-cell rules of a
 * staggered grid (boundary on the cell face):
 *     periodic  p_0 = p_n, p_{n+1} = p_1
 *     Neumann   p_0 = p_1          (and p_{n+1} = p_n)
 *     Dirichlet p_0 = -p_1         (and p_{n+1} = -p_n)
 * and are pinned by the test suite against brute-force eigendecompositions
 * and textbook DCT/DST/DFT routines.
 *
 * Everything is computed in REAL, which is double unless this file is
 * compiled with -DORACLE_LONG_DOUBLE (x86 80-bit extended), the error-bound
 * variant.  Interfaces always take and return double.
 *
 * Layout: every 3-D field is x fastest, a[i + nx*(j + ny*k)].
 * Boundary codes per face: 0 = periodic, 1 = Neumann, 2 = Dirichlet;
 * bc[6] = {x-, x+, y-, y+, z-, z+}.  Codes 3 and 4 describe a field that
 * lives on the cell faces of an axis instead of the cell centres (a velocity
 * component along its own direction, as in the implicit diffusion steps of
 * eq. (up_id_2)); both ends of such an axis carry 3 or 4:
 *   3  Dirichlet on the boundary face: the field is zero there and the face
 *      is not an unknown;
 *   4  Neumann on the boundary face: the face is an unknown, and the zero
 *      derivative across it mirrors the field about it (w_{-1} = w_1).
 * Along x or y with C cells of width h the unknowns are therefore the C-1
 * interior faces (3,3), all C+1 faces (4,4), or the C faces other than the
 * Dirichlet one ((3,4), (4,3)); the operator is (w_{i-1} - 2 w_i +
 * w_{i+1})/h^2.  Along z only (3,3) is allowed: the unknowns are the nz
 * interior faces of a grid of nz+1 cells, dzf then holds those nz+1 cell
 * widths (stretched), and the operator is the flux form of zcoef_real.
 */
#include <math.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>

#ifdef ORACLE_LONG_DOUBLE
typedef long double REAL;
#define RCOS cosl
#define RSIN sinl
#define RPI 3.141592653589793238462643383279502884L
#define SYM(name) name##_ld
#else
typedef double REAL;
#define RCOS cos
#define RSIN sin
#define RPI 3.141592653589793238462643383279502884
#define SYM(name) name
#endif

enum { BC_P = 0, BC_N = 1, BC_D = 2, BC_DF = 3, BC_NF = 4 };

/* Threads of the OpenMP loops below (for timing the oracle on n cores), and
 * the number a parallel loop will use. */
void SYM(oracle_set_threads)(int n) { omp_set_num_threads(n > 0 ? n : 1); }
int SYM(oracle_threads)(void) { return omp_get_max_threads(); }
/* transform kinds of one axis, named by the (lower, upper) boundary pair;
 * K_FD .. K_FND are the face-located pairs (3,3), (4,4), (3,4), (4,3) */
enum { K_P = 0, K_NN = 1, K_DD = 2, K_ND = 3, K_DN = 4, K_FD = 5, K_FN = 6, K_FDN = 7, K_FND = 8 };

static int is_face(int code) { return code == BC_DF || code == BC_NF; }

/* Axis kind from its two face conditions; -1 when the pair is invalid
 * (periodic must be paired with periodic, a face-located field has code 3
 * or 4 at both ends). */
int SYM(oracle_axis_kind)(int lo, int hi)
{
    if (is_face(lo) || is_face(hi)) {
        if (!is_face(lo) || !is_face(hi)) return -1;
        if (lo == BC_DF) return hi == BC_DF ? K_FD : K_FDN;
        return hi == BC_NF ? K_FN : K_FND;
    }
    if (lo == BC_P || hi == BC_P) return (lo == BC_P && hi == BC_P) ? K_P : -1;
    if (lo == BC_N && hi == BC_N) return K_NN;
    if (lo == BC_D && hi == BC_D) return K_DD;
    if (lo == BC_N && hi == BC_D) return K_ND;
    if (lo == BC_D && hi == BC_N) return K_DN;
    return -1;
}

/*
 * Eigenvector rows and eigenvalues mu[q] of the 1-D operator (p_{i-1} - 2 p_i
 * + p_{i+1}) with the ghost rules above (unit spacing).  These are the
 * discrete transforms F of Section 2.  R[q][i] (row-major, R[q*n+i]) is the
 * q-th eigenvector of the operator (A R_q = mu_q R_q), T[q][i] = w_i R[q][i]
 * the q-th row of the forward transform (T A = diag(mu) T), with w_i = 1/2
 * on an unknown that sits on a Neumann boundary face (codes 4) and 1
 * elsewhere, so that T is the left eigenvector matrix (w A is symmetric).
 * Cell-centred kinds (w = 1, T = R):
 *   P : real DFT, stored in the order
 *       q=0: 1,  q=1: (-1)^i,  q=2l: cos(2 pi l i/n),  q=2l+1: -sin(2 pi l i/n)
 *       (l = 1..n/2-1; for odd n the (-1)^i row does not exist and the pairs
 *       run l = 1..(n-1)/2 from q = 1), mu = -4 sin^2(pi l/n);
 *   NN: cos(pi q (i+1/2)/n)            DCT-II,  mu = -4 sin^2(pi q/(2n));
 *   DD: sin(pi (q+1)(i+1/2)/n)         DST-II,  mu = -4 sin^2(pi (q+1)/(2n));
 *   ND: cos(pi (2q+1)(2i+1)/(4n))      DCT-IV,  mu = -4 sin^2(pi (2q+1)/(4n));
 *   DN: sin(pi (2q+1)(2i+1)/(4n))      DST-IV,  mu as ND.
 * Face-located kinds (unknown i on a face; R, and the weighted T):
 *   FD : sin(pi (q+1)(i+1)/(n+1))      DST-I,   mu = -4 sin^2(pi (q+1)/(2(n+1)));
 *   FN : cos(pi q i/(n-1))             DCT-I,   mu = -4 sin^2(pi q/(2(n-1))),
 *        w_0 = w_{n-1} = 1/2 (n >= 2);
 *   FDN: sin(pi (2q+1)(i+1)/(2n))      DST-III-type, mu = -4 sin^2(pi (2q+1)/(4n)),
 *        w_{n-1} = 1/2;
 *   FND: cos(pi (2q+1) i/(2n))         DCT-III-type, mu as FDN, w_0 = 1/2.
 */
static REAL face_weight(int kind, int n, int i)
{
    if ((kind == K_FN && (i == 0 || i == n - 1)) || (kind == K_FDN && i == n - 1) || (kind == K_FND && i == 0))
        return (REAL)0.5;
    return 1;
}

static void eigen_real(int kind, int n, REAL *T, REAL *R, REAL *mu)
{
    for (int q = 0; q < n; ++q) {
        REAL wav = 0; /* the angle whose sin^2 gives mu */
        for (int i = 0; i < n; ++i) {
            REAL v = 0, x = (REAL)i + (REAL)0.5;
            switch (kind) {
            case K_P: {
                int l, is_sin = 0;
                if (q == 0) l = 0;
                else if (n % 2 == 0 && q == 1) l = n / 2;
                else if (n % 2 == 0) { l = q / 2; is_sin = q & 1; }
                else { l = (q + 1) / 2; is_sin = !(q & 1); }
                REAL ang = 2 * RPI * (REAL)l * (REAL)i / (REAL)n;
                v = is_sin ? -RSIN(ang) : RCOS(ang);
                if (n % 2 == 0 && q == 1) v = (i & 1) ? -1 : 1;
                wav = RPI * (REAL)l / (REAL)n;
                break;
            }
            case K_NN: v = RCOS(RPI * (REAL)q * x / (REAL)n); wav = RPI * (REAL)q / (2 * (REAL)n); break;
            case K_DD: v = RSIN(RPI * (REAL)(q + 1) * x / (REAL)n); wav = RPI * (REAL)(q + 1) / (2 * (REAL)n); break;
            case K_ND: v = RCOS(RPI * (REAL)(2 * q + 1) * (2 * x) / (4 * (REAL)n)); wav = RPI * (REAL)(2 * q + 1) / (4 * (REAL)n); break;
            case K_DN: v = RSIN(RPI * (REAL)(2 * q + 1) * (2 * x) / (4 * (REAL)n)); wav = RPI * (REAL)(2 * q + 1) / (4 * (REAL)n); break;
            case K_FD:
                v = RSIN(RPI * (REAL)(q + 1) * (REAL)(i + 1) / (REAL)(n + 1));
                wav = RPI * (REAL)(q + 1) / (2 * (REAL)(n + 1));
                break;
            case K_FN:
                v = RCOS(RPI * (REAL)q * (REAL)i / (REAL)(n - 1));
                wav = RPI * (REAL)q / (2 * (REAL)(n - 1));
                break;
            case K_FDN:
                v = RSIN(RPI * (REAL)(2 * q + 1) * (REAL)(i + 1) / (2 * (REAL)n));
                wav = RPI * (REAL)(2 * q + 1) / (4 * (REAL)n);
                break;
            case K_FND:
                v = RCOS(RPI * (REAL)(2 * q + 1) * (REAL)i / (2 * (REAL)n));
                wav = RPI * (REAL)(2 * q + 1) / (4 * (REAL)n);
                break;
            }
            if (R) R[(size_t)q * n + i] = v;
            T[(size_t)q * n + i] = face_weight(kind, n, i) * v;
        }
        REAL s = RSIN(wav);
        mu[q] = -4 * s * s;
    }
}

void SYM(oracle_eigen)(int kind, int n, double *T, double *mu)
{
    REAL *Tr = malloc(sizeof(REAL) * (size_t)n * n), *mr = malloc(sizeof(REAL) * n);
    eigen_real(kind, n, Tr, NULL, mr);
    for (size_t e = 0; e < (size_t)n * n; ++e) T[e] = (double)Tr[e];
    for (int q = 0; q < n; ++q) mu[q] = (double)mr[q];
    free(Tr); free(mr);
}

/* Index of the constant (zero-eigenvalue) row of an axis, or -1 if none.
 * P, NN and FN have one, and it is row 0 in every order above. */
static int zero_row(int kind) { return (kind == K_P || kind == K_NN || kind == K_FN) ? 0 : -1; }

/* An x or y axis of n unknowns: a valid kind, and at least two unknowns when
 * one of its ends is a Neumann face (the mirror needs the second face). */
static int axis_ok(int kind, int n)
{
    if (kind < 0) return 0;
    if (kind == K_FN || kind == K_FDN || kind == K_FND) return n >= 2;
    return 1;
}

/*
 * Tridiagonal coefficients of the z operator, conservative form
 *   [(p_{k+1}-p_k)/dzc_k - (p_k-p_{k-1})/dzc_{k-1}] / dzf_k
 * with dzc_k = (dzf_k + dzf_{k+1})/2 between cells and a mirror ghost cell at
 * a wall (dzc = dzf of the wall cell).  Row k reads
 *   a[k] p_{k-1} + b[k] p_k + c[k] p_{k+1}.
 * Periodic: the corner entries a[0] (couples to p_{nz-1}) and c[nz-1]
 * (couples to p_0) are kept.  Wall rows fold the ghost into the diagonal and
 * zero the outer coefficient.  Returns 0, or -1 on an invalid pair.
 *
 * Face-located field (code 3 at both ends): unknown k sits on the face
 * between cells k and k+1 of a grid of nz+1 cells with widths dzf[0..nz].
 * The neighbouring unknowns are dzf[k] below and dzf[k+1] above, and the
 * control volume reaches from the centre of cell k to that of cell k+1:
 *   [(w_{k+1}-w_k)/dzf_{k+1} - (w_k-w_{k-1})/dzf_k] / ((dzf_k + dzf_{k+1})/2).
 * The two wall faces hold w = 0, so their couplings drop out of the end rows
 * while the diagonal keeps both terms.
 */
static int zcoef_real(int nz, int lo, int hi, const double *dzf, REAL *a, REAL *b, REAL *c)
{
    int kz = SYM(oracle_axis_kind)(lo, hi);
    if (kz < 0 || kz > K_FD) return -1;  /* of the face-located pairs z takes (3,3) only */
    if (lo == BC_DF) {
        for (int k = 0; k < nz; ++k) {
            REAL below = dzf[k], above = dzf[k + 1], cv = (below + above) / 2;
            a[k] = 1 / (below * cv);
            c[k] = 1 / (above * cv);
            b[k] = -(a[k] + c[k]);
        }
        a[0] = 0;
        c[nz - 1] = 0;
        return 0;
    }
    for (int k = 0; k < nz; ++k) {
        REAL f = dzf[k], cm, cp;
        if (k > 0) cm = ((REAL)dzf[k - 1] + f) / 2;
        else cm = (lo == BC_P) ? ((REAL)dzf[nz - 1] + f) / 2 : f;
        if (k < nz - 1) cp = (f + (REAL)dzf[k + 1]) / 2;
        else cp = (hi == BC_P) ? (f + (REAL)dzf[0]) / 2 : f;
        a[k] = 1 / (cm * f);
        c[k] = 1 / (cp * f);
        b[k] = -(a[k] + c[k]);
    }
    if (lo == BC_N) { b[0] += a[0]; a[0] = 0; }
    if (lo == BC_D) { b[0] -= a[0]; a[0] = 0; }
    if (hi == BC_N) { b[nz - 1] += c[nz - 1]; c[nz - 1] = 0; }
    if (hi == BC_D) { b[nz - 1] -= c[nz - 1]; c[nz - 1] = 0; }
    return 0;
}

int SYM(oracle_zcoef)(int nz, int lo, int hi, const double *dzf, double *a, double *b, double *c)
{
    REAL *ar = malloc(sizeof(REAL) * 3 * nz);
    int rc = zcoef_real(nz, lo, hi, dzf, ar, ar + nz, ar + 2 * nz);
    for (int k = 0; k < nz && rc == 0; ++k) { a[k] = (double)ar[k]; b[k] = (double)ar[nz + k]; c[k] = (double)ar[2 * nz + k]; }
    free(ar);
    return rc;
}

/* Gauss elimination without pivoting on a tridiagonal system (Thomas):
 * forward elimination of the sub-diagonal, then back substitution.
 * a[0] and c[n-1] are ignored.  w is scratch of length n. */
static void thomas(int n, const REAL *a, const REAL *b, const REAL *c, const REAL *d, REAL *x, REAL *w)
{
    REAL piv = b[0];
    x[0] = d[0] / piv;
    for (int k = 1; k < n; ++k) {
        w[k] = c[k - 1] / piv;
        piv = b[k] - a[k] * w[k];
        x[k] = (d[k] - a[k] * x[k - 1]) / piv;
    }
    for (int k = n - 2; k >= 0; --k) x[k] -= w[k + 1] * x[k + 1];
}

/* Periodic (cyclic) tridiagonal system by the Sherman-Morrison formula:
 * A = A' + u v^T with u = (g, 0..0, c[n-1]), v = (1, 0..0, a[0]/g), g = -b[0];
 * solve A' y = d and A' z = u, then x = y - z (v.y)/(1 + v.z).
 * w is scratch of length 4n.  Requires n >= 3. */
static void thomas_cyclic(int n, const REAL *a, const REAL *b, const REAL *c, const REAL *d, REAL *x, REAL *w)
{
    REAL *bb = w, *u = w + n, *z = w + 2 * n, *s = w + 3 * n;
    REAL g = -b[0];
    for (int k = 0; k < n; ++k) { bb[k] = b[k]; u[k] = 0; }
    bb[0] = b[0] - g;
    bb[n - 1] = b[n - 1] - c[n - 1] * a[0] / g;
    u[0] = g; u[n - 1] = c[n - 1];
    thomas(n, a, bb, c, d, x, s);
    thomas(n, a, bb, c, u, z, s);
    REAL vy = x[0] + a[0] / g * x[n - 1];
    REAL vz = z[0] + a[0] / g * z[n - 1];
    REAL fac = vy / (1 + vz);
    for (int k = 0; k < n; ++k) x[k] -= fac * z[k];
}

void SYM(oracle_tridiag)(int n, const double *a, const double *b, const double *c, const double *d, double *x, int cyclic)
{
    REAL *r = malloc(sizeof(REAL) * 10 * (size_t)n);
    REAL *ar = r, *br = r + n, *cr = r + 2 * n, *dr = r + 3 * n, *xr = r + 4 * n, *wr = r + 5 * n;
    for (int k = 0; k < n; ++k) { ar[k] = a[k]; br[k] = b[k]; cr[k] = c[k]; dr[k] = d[k]; }
    if (cyclic) thomas_cyclic(n, ar, br, cr, dr, xr, wr);
    else thomas(n, ar, br, cr, dr, xr, wr);
    for (int k = 0; k < n; ++k) x[k] = (double)xr[k];
    free(r);
}

/* ------------------------------------------------------------------------ */
/* Transforms along one axis of a REAL field: out = M applied along `axis`,  */
/* where M is an n x n matrix (row-major).  Summation runs i = 0..n-1.       */
static void apply_along(int axis, int nx, int ny, int nz, const REAL *M, const REAL *in, REAL *out)
{
    if (axis == 0) {
        #pragma omp parallel for schedule(static)
        for (long line = 0; line < (long)ny * nz; ++line) {
            const REAL *src = in + line * nx;
            REAL *dst = out + line * nx;
            for (int q = 0; q < nx; ++q) {
                REAL s = 0;
                for (int i = 0; i < nx; ++i) s += M[(size_t)q * nx + i] * src[i];
                dst[q] = s;
            }
        }
    } else if (axis == 1) {
        #pragma omp parallel for schedule(static)
        for (long kq = 0; kq < (long)nz * ny; ++kq) {
            long k = kq / ny; int q = (int)(kq % ny);
            REAL *dst = out + (size_t)nx * (q + (size_t)ny * k);
            for (int i = 0; i < nx; ++i) dst[i] = 0;
            for (int j = 0; j < ny; ++j) {
                REAL m = M[(size_t)q * ny + j];
                const REAL *src = in + (size_t)nx * (j + (size_t)ny * k);
                for (int i = 0; i < nx; ++i) dst[i] += m * src[i];
            }
        }
    } else {
        size_t plane = (size_t)nx * ny;
        #pragma omp parallel for schedule(static)
        for (long kq = 0; kq < (long)nz; ++kq) {
            REAL *dst = out + plane * kq;
            for (size_t e = 0; e < plane; ++e) dst[e] = 0;
            for (int k = 0; k < nz; ++k) {
                REAL m = M[(size_t)kq * nz + k];
                const REAL *src = in + plane * k;
                for (size_t e = 0; e < plane; ++e) dst[e] += m * src[e];
            }
        }
    }
}

/* Forward matrix T and its inverse T^{-1}[i][q] = R[q][i] / (T_q . R_q):
 * the left and right eigenvectors of one operator are biorthogonal
 * (T_q . R_p = 0 for mu_q != mu_p; the repeated eigenvalues of P come in
 * sin/cos pairs, orthogonal too), so T R^T is diagonal and its diagonal,
 * computed by a plain sum, normalises the inverse.  With w = 1 (the
 * cell-centred kinds) this is T^T diag(1/|row_q|^2). */
static void forward_inverse(int kind, int n, REAL *T, REAL *Ti, REAL *mu)
{
    REAL *R = malloc(sizeof(REAL) * (size_t)n * n);
    eigen_real(kind, n, T, R, mu);
    for (int q = 0; q < n; ++q) {
        REAL nn = 0;
        for (int i = 0; i < n; ++i) nn += T[(size_t)q * n + i] * R[(size_t)q * n + i];
        for (int i = 0; i < n; ++i) Ti[(size_t)i * n + q] = R[(size_t)q * n + i] / nn;
    }
    free(R);
}

static REAL *to_real(const double *v, size_t n)
{
    REAL *r = malloc(sizeof(REAL) * n);
    for (size_t e = 0; e < n; ++e) r[e] = v[e];
    return r;
}
static void from_real(const REAL *r, double *v, size_t n)
{
    for (size_t e = 0; e < n; ++e) v[e] = (double)r[e];
}

/* Public: out = T (inverse = 0) or T^{-1} (inverse = 1) of `kind` along axis. */
void SYM(oracle_transform)(int axis, int inverse, int kind, int nx, int ny, int nz, const double *in, double *out)
{
    int n = axis == 0 ? nx : axis == 1 ? ny : nz;
    size_t N = (size_t)nx * ny * nz;
    REAL *T = malloc(sizeof(REAL) * (size_t)n * n), *Ti = malloc(sizeof(REAL) * (size_t)n * n), *mu = malloc(sizeof(REAL) * n);
    forward_inverse(kind, n, T, Ti, mu);
    REAL *a = to_real(in, N), *b = malloc(sizeof(REAL) * N);
    apply_along(axis, nx, ny, nz, inverse ? Ti : T, a, b);
    from_real(b, out, N);
    free(T); free(Ti); free(mu); free(a); free(b);
}

/*
 * Solve the tridiagonal systems of eq. (poi_reduced) for every (i,j) column
 * of a spectral field fh (x and y already transformed), in place.
 *   lambda(i,j) = mu_x(i)/dx^2 + mu_y(j)/dy^2 + shift is added to the z
 *   diagonal (shift: the Helmholtz form (L_h + shift) p = f of implicit
 *   diffusion, the same expansion with the diagonal moved; shift <= 0).
 * Singular column: all three axes are P or NN and (i,j) is the constant row
 * of both x and y.  Then the column is projected onto the range
 * (fh_k -= sum_k w_k fh_k / sum_k w_k, w = dzf, the left null vector of the
 * z operator), solved with its last equation replaced by p_{nz-1} = 0, and
 * shifted to zero dzf-weighted mean.  The removed weighted mean of the
 * spectral column is returned in *removed (0 when nothing is singular).
 */
static int spectral_solve_real(int nx, int ny, int nz, const int bc[6], double dx, double dy,
                               const double *dzf, double shift, REAL *fh, REAL *removed)
{
    int kx = SYM(oracle_axis_kind)(bc[0], bc[1]), ky = SYM(oracle_axis_kind)(bc[2], bc[3]);
    int kz = SYM(oracle_axis_kind)(bc[4], bc[5]);
    if (!axis_ok(kx, nx) || !axis_ok(ky, ny) || kz < 0 || kz > K_FD) return -1;
    /* a face-located Neumann pair (DCT-I) has a constant mode too; a problem
     * it would make singular is not defined here */
    if ((kz == K_P || kz == K_NN) && shift == 0.0 && zero_row(kx) >= 0 && zero_row(ky) >= 0 &&
        (kx == K_FN || ky == K_FN))
        return -1;
    REAL *T = malloc(sizeof(REAL) * ((size_t)nx * nx + (size_t)ny * ny));
    REAL *mux = malloc(sizeof(REAL) * (nx + ny)), *muy = mux + nx;
    eigen_real(kx, nx, T, NULL, mux);
    eigen_real(ky, ny, T + (size_t)nx * nx, NULL, muy);
    REAL *za = malloc(sizeof(REAL) * 3 * nz), *zb = za + nz, *zc = za + 2 * nz;
    zcoef_real(nz, bc[4], bc[5], dzf, za, zb, zc);
    int zx = zero_row(kx), zy = zero_row(ky);
    /* a nonzero shift (Helmholtz) leaves no singular column */
    int z_singular = (kz == K_P || kz == K_NN) && shift == 0.0;
    int cyclic = (kz == K_P);
    REAL wsum = 0;
    for (int k = 0; k < nz; ++k) wsum += dzf[k];
    *removed = 0;
    size_t plane = (size_t)nx * ny;
    #pragma omp parallel
    {
        REAL *d = malloc(sizeof(REAL) * 16 * (size_t)(nz + 2));
        REAL *x = d + (nz + 2), *bb = d + 2 * (nz + 2), *w = d + 3 * (nz + 2);
        #pragma omp for schedule(static)
        for (long col = 0; col < (long)plane; ++col) {
            int i = (int)(col % nx), j = (int)(col / nx);
            REAL lam = mux[i] / ((REAL)dx * dx) + muy[j] / ((REAL)dy * dy) + (REAL)shift;
            for (int k = 0; k < nz; ++k) { d[k] = fh[col + plane * k]; bb[k] = zb[k] + lam; }
            int singular = z_singular && i == zx && j == zy;
            if (singular) {
                REAL s = 0;
                for (int k = 0; k < nz; ++k) s += (REAL)dzf[k] * d[k];
                REAL m = s / wsum;
                *removed = m;
                for (int k = 0; k < nz; ++k) d[k] -= m;
                if (nz == 1) {
                    x[0] = 0;
                } else {
                    /* last equation replaced by p_{nz-1} = 0; the periodic
                     * corner couplings then multiply the pinned unknown */
                    REAL *aa = w + 6 * (nz + 2), *cc = w + 7 * (nz + 2);
                    for (int k = 0; k < nz; ++k) { aa[k] = za[k]; cc[k] = zc[k]; }
                    aa[0] = 0;
                    aa[nz - 1] = 0; bb[nz - 1] = 1; d[nz - 1] = 0;
                    thomas(nz, aa, bb, cc, d, x, w);
                }
                REAL s2 = 0;
                for (int k = 0; k < nz; ++k) s2 += (REAL)dzf[k] * x[k];
                REAL m2 = s2 / wsum;
                for (int k = 0; k < nz; ++k) x[k] -= m2;
            } else if (cyclic && nz >= 3) {
                thomas_cyclic(nz, za, bb, zc, d, x, w);
            } else if (cyclic) {
                /* nz = 1 or 2: the periodic couplings fold onto the same or
                 * the other cell; write the small system out directly */
                if (nz == 1) x[0] = d[0] / lam;
                else {
                    REAL a11 = bb[0], a12 = za[0] + zc[0], a21 = za[1] + zc[1], a22 = bb[1];
                    REAL det = a11 * a22 - a12 * a21;
                    x[0] = (a22 * d[0] - a12 * d[1]) / det;
                    x[1] = (a11 * d[1] - a21 * d[0]) / det;
                }
            } else {
                thomas(nz, za, bb, zc, d, x, w);
            }
            for (int k = 0; k < nz; ++k) fh[col + plane * k] = x[k];
        }
        free(d);
    }
    free(T); free(mux); free(za);
    return 0;
}

int SYM(oracle_spectral_solve)(int nx, int ny, int nz, const int bc[6], double dx, double dy,
                               const double *dzf, double shift, const double *fh, double *ph, double *removed)
{
    size_t N = (size_t)nx * ny * nz;
    REAL *a = to_real(fh, N), rem = 0;
    int rc = spectral_solve_real(nx, ny, nz, bc, dx, dy, dzf, shift, a, &rem);
    from_real(a, ph, N);
    if (removed) *removed = (double)rem;
    free(a);
    return rc;
}

/*
 * The whole solve: p = T_x^{-1} T_y^{-1} S (T_y T_x f), where S is the
 * column-wise tridiagonal solve above.  info[0] receives the removed
 * dzf-weighted mean of f in physical units (0 when the problem is not
 * singular); it is the spectral value divided by nx*ny, because the constant
 * rows of P and NN are all ones.
 */
int SYM(oracle_solve)(int nx, int ny, int nz, const int bc[6], double dx, double dy,
                      const double *dzf, double shift, const double *f, double *p, double *info)
{
    int kx = SYM(oracle_axis_kind)(bc[0], bc[1]), ky = SYM(oracle_axis_kind)(bc[2], bc[3]);
    int kz = SYM(oracle_axis_kind)(bc[4], bc[5]);
    if (!axis_ok(kx, nx) || !axis_ok(ky, ny) || kz < 0 || kz > K_FD) return -1;
    if ((kz == K_P || kz == K_NN) && shift == 0.0 && zero_row(kx) >= 0 && zero_row(ky) >= 0 &&
        (kx == K_FN || ky == K_FN))
        return -1;
    size_t N = (size_t)nx * ny * nz;
    REAL *Tx = malloc(sizeof(REAL) * (size_t)nx * nx), *Tix = malloc(sizeof(REAL) * (size_t)nx * nx);
    REAL *Ty = malloc(sizeof(REAL) * (size_t)ny * ny), *Tiy = malloc(sizeof(REAL) * (size_t)ny * ny);
    REAL *mu = malloc(sizeof(REAL) * (nx > ny ? nx : ny));
    forward_inverse(kx, nx, Tx, Tix, mu);
    forward_inverse(ky, ny, Ty, Tiy, mu);
    REAL *a = to_real(f, N), *b = malloc(sizeof(REAL) * N), rem = 0;
    apply_along(0, nx, ny, nz, Tx, a, b);
    apply_along(1, nx, ny, nz, Ty, b, a);
    int rc = spectral_solve_real(nx, ny, nz, bc, dx, dy, dzf, shift, a, &rem);
    apply_along(1, nx, ny, nz, Tiy, a, b);
    apply_along(0, nx, ny, nz, Tix, b, a);
    from_real(a, p, N);
    if (info) info[0] = (double)(rem / ((REAL)nx * ny));
    free(Tx); free(Tix); free(Ty); free(Tiy); free(mu); free(a); free(b);
    return rc;
}

/*
 * out = L_h p + shift p, the 7-point operator of eq. (poi) with the z part
 * in the conservative form above and the ghost rules of each face (a
 * face-located z field: the form of zcoef_real, zero on the wall faces; a
 * face-located x or y field: the rules of codes 3 and 4 in the header).
 * Boundary codes are taken as given (x and y need nx, ny >= 2 for code 4).
 */
void SYM(oracle_apply_L)(int nx, int ny, int nz, const int bc[6], double dx, double dy,
                         const double *dzf, double shift, const double *p, double *out)
{
    REAL *zaf = malloc(sizeof(REAL) * 2 * nz), *zcf = zaf + nz;
    /* full (unfolded) z coefficients: a/c before the ghost is folded in */
    for (int k = 0; k < nz; ++k) {
        REAL f = dzf[k], cm, cp;
        cm = k > 0 ? ((REAL)dzf[k - 1] + f) / 2 : (bc[4] == BC_P ? ((REAL)dzf[nz - 1] + f) / 2 : f);
        cp = k < nz - 1 ? (f + (REAL)dzf[k + 1]) / 2 : (bc[5] == BC_P ? (f + (REAL)dzf[0]) / 2 : f);
        zaf[k] = 1 / (cm * f);
        zcf[k] = 1 / (cp * f);
        if (bc[4] == BC_DF) {
            REAL below = dzf[k], above = dzf[k + 1], cv = (below + above) / 2;
            zaf[k] = 1 / (below * cv);
            zcf[k] = 1 / (above * cv);
        }
    }
    REAL ix2 = 1 / ((REAL)dx * dx), iy2 = 1 / ((REAL)dy * dy);
    #pragma omp parallel for schedule(static)
    for (long kj = 0; kj < (long)nz * ny; ++kj) {
        int k = (int)(kj / ny), j = (int)(kj % ny);
        for (int i = 0; i < nx; ++i) {
#define P3(ii, jj, kk) ((REAL)p[(ii) + (size_t)nx * ((jj) + (size_t)ny * (kk))])
            REAL c0 = P3(i, j, k);
            /* neighbour value through the ghost rule of a face */
            REAL xm, xp, ym, yp, zm, zp;
            /* x and y: a face-located field is zero beyond a Dirichlet face
             * (code 3) and mirrored about a Neumann face it sits on (code 4) */
            xm = i > 0 ? P3(i - 1, j, k) : bc[0] == BC_P ? P3(nx - 1, j, k) : bc[0] == BC_N ? c0
                 : bc[0] == BC_DF ? 0 : bc[0] == BC_NF ? P3(1, j, k) : -c0;
            xp = i < nx - 1 ? P3(i + 1, j, k) : bc[1] == BC_P ? P3(0, j, k) : bc[1] == BC_N ? c0
                 : bc[1] == BC_DF ? 0 : bc[1] == BC_NF ? P3(nx - 2, j, k) : -c0;
            ym = j > 0 ? P3(i, j - 1, k) : bc[2] == BC_P ? P3(i, ny - 1, k) : bc[2] == BC_N ? c0
                 : bc[2] == BC_DF ? 0 : bc[2] == BC_NF ? P3(i, 1, k) : -c0;
            yp = j < ny - 1 ? P3(i, j + 1, k) : bc[3] == BC_P ? P3(i, 0, k) : bc[3] == BC_N ? c0
                 : bc[3] == BC_DF ? 0 : bc[3] == BC_NF ? P3(i, ny - 2, k) : -c0;
            zm = k > 0 ? P3(i, j, k - 1) : bc[4] == BC_P ? P3(i, j, nz - 1) : bc[4] == BC_N ? c0
                 : bc[4] == BC_DF ? 0 : -c0;
            zp = k < nz - 1 ? P3(i, j, k + 1) : bc[5] == BC_P ? P3(i, j, 0) : bc[5] == BC_N ? c0
                 : bc[5] == BC_DF ? 0 : -c0;
#undef P3
            REAL v = (xm - 2 * c0 + xp) * ix2 + (ym - 2 * c0 + yp) * iy2
                   + zcf[k] * (zp - c0) - zaf[k] * (c0 - zm) + (REAL)shift * c0;
            out[i + (size_t)nx * (j + (size_t)ny * k)] = (double)v;
        }
    }
    free(zaf);
}

/*
 * Plain CPU reference ("oracle") for the spectrally truncated four-wave
 * collision operator of Qi, Shen and Wang, "A fast Fourier spectral method
 * for wave kinetic equation" (arXiv 2503.12805).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code with
 * the GPU path and uses no FFT anywhere: every transform is a direct sum in
 * IEEE double precision, evaluated in a fixed order (results do not depend
 * on the OpenMP thread count).
 *
 * Conventions (readings of the paper where it is silent):
 *   - grid node x in {0..N-1} per axis sits at k = -L + h x, h = 2L/N;
 *   - Fourier arrays are stored in FFT index order: slot i holds the signed
 *     mode j(i) = i for i < N/2 and i - N otherwise, so slot N/2 is the mode
 *     -N/2, which the truncated series of eq. (fj) keeps;
 *   - multi-dimensional arrays are row-major, last axis fastest, complex
 *     values interleaved (re, im);
 *   - the discrete convolutions of Alg. 1 are cyclic (mode sums wrap mod N)
 *     unless the caller asks for the exact-Galerkin ("linear") constraint
 *     l + m + n = j of eq. (KK1).
 *
 * Parity status per function is stated in each header comment.
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

#define ORACLE_OK 0
#define ORACLE_ERR_INVALID (-1)
#define ORACLE_ERR_NOMEM (-4)

static int signed_mode(int i, int N) { return i < N / 2 ? i : i - N; }

static int ipow(int b, int e) { int r = 1; while (e-- > 0) r *= b; return r; }

/* ------------------------------------------------------------------------ */
/* Quadrature (eq. (G1): Gauss-Legendre in |q|; midpoint rule on the circle  */
/* in 2D; closed-form spherical designs on S^2 in 3D).                        */
/* ------------------------------------------------------------------------ */

/* n-point Gauss-Legendre rule on [-1, 1], nodes ascending.  Each root of
 * P_n is found by Newton's method on the three-term recurrence
 * (k+1) P_{k+1} = (2k+1) x P_k - k P_{k-1}; the weight is
 * 2 / ((1 - x^2) P_n'(x)^2).  Pinned against numpy's leggauss and against
 * exact polynomial integrals in the tests. */
int oracle_gauss_legendre(int n, double *t, double *w)
{
    if (n < 1 || !t || !w) return ORACLE_ERR_INVALID;
    for (int i = 0; i < n; ++i) {
        /* standard initial guess for the (i+1)-th largest root */
        double x = cos(M_PI * (i + 0.75) / (n + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = x;
            if (n == 1) { p1 = x; p0 = 1.0; }
            for (int k = 1; k < n; ++k) {
                double p2 = ((2.0 * k + 1.0) * x * p1 - k * p0) / (k + 1.0);
                p0 = p1; p1 = p2;
            }
            /* p1 = P_n(x), p0 = P_{n-1}(x) */
            dp = n * (x * p1 - p0) / (x * x - 1.0);
            double dx = p1 / dp;
            x -= dx;
            if (fabs(dx) <= 1e-16 * (1.0 + fabs(x))) break;
        }
        /* recompute derivative at the converged root */
        {
            double p0 = 1.0, p1 = x;
            for (int k = 1; k < n; ++k) {
                double p2 = ((2.0 * k + 1.0) * x * p1 - k * p0) / (k + 1.0);
                p0 = p1; p1 = p2;
            }
            dp = n * (x * p1 - p0) / (x * x - 1.0);
        }
        /* roots come out descending; store ascending */
        t[n - 1 - i] = x;
        w[n - 1 - i] = 2.0 / ((1.0 - x * x) * dp * dp);
    }
    return ORACLE_OK;
}

/* Sphere rules, unnormalised measure (weights sum to |S^{d-1}|).
 *   d = 2, rule 0: midpoint rule, angle (2i+1) pi / n, weight 2 pi / n.
 *   d = 3, rule 1: octahedron, the 6 points +-e_a (a spherical 3-design).
 *          rule 2: cube, the 8 points (+-1,+-1,+-1)/sqrt 3 (3-design).
 *          rule 3: icosahedron, the 12 vertices, cyclic permutations of
 *                  (0, +-1, +-phi)/sqrt(1+phi^2) (5-design).
 * Weights are equal, 4 pi / n.  Returns the point count, or an error. */
int oracle_sphere_rule(int d, int rule, int n, double *pts, double *w)
{
    if (!pts || !w) return ORACLE_ERR_INVALID;
    if (d == 2) {
        if (rule != 0 || n < 1) return ORACLE_ERR_INVALID;
        for (int i = 0; i < n; ++i) {
            double th = (2.0 * i + 1.0) * M_PI / n;
            pts[2 * i] = cos(th);
            pts[2 * i + 1] = sin(th);
            w[i] = 2.0 * M_PI / n;
        }
        return n;
    }
    if (d != 3) return ORACLE_ERR_INVALID;
    int cnt = 0;
    if (rule == 1) {
        if (n != 6) return ORACLE_ERR_INVALID;
        for (int a = 0; a < 3; ++a)
            for (int s = 0; s < 2; ++s) {
                double *p = pts + 3 * cnt++;
                p[0] = p[1] = p[2] = 0.0;
                p[a] = s ? -1.0 : 1.0;
            }
    } else if (rule == 2) {
        if (n != 8) return ORACLE_ERR_INVALID;
        double c = 1.0 / sqrt(3.0);
        for (int i = 0; i < 8; ++i) {
            double *p = pts + 3 * cnt++;
            p[0] = (i & 4) ? -c : c;
            p[1] = (i & 2) ? -c : c;
            p[2] = (i & 1) ? -c : c;
        }
    } else if (rule == 3) {
        if (n != 12) return ORACLE_ERR_INVALID;
        double phi = 0.5 * (1.0 + sqrt(5.0));
        double nrm = sqrt(1.0 + phi * phi);
        for (int cyc = 0; cyc < 3; ++cyc)
            for (int s1 = 0; s1 < 2; ++s1)
                for (int s2 = 0; s2 < 2; ++s2) {
                    double v[3] = {0.0, s1 ? -1.0 : 1.0, s2 ? -phi : phi};
                    double *p = pts + 3 * cnt++;
                    for (int a = 0; a < 3; ++a) p[(a + cyc) % 3] = v[a] / nrm;
                }
    } else {
        return ORACLE_ERR_INVALID;
    }
    for (int i = 0; i < n; ++i) w[i] = 4.0 * M_PI / n;
    return n;
}

/* ------------------------------------------------------------------------ */
/* Separable direct sums along one axis of an N^d complex array.             */
/* out[.., y, ..] = sum_x mat[y*N + x] in[.., x, ..] along axis `axis`.       */
/* ------------------------------------------------------------------------ */
static void apply_axis(int d, int N, int axis, const cplx *mat, const cplx *in, cplx *out)
{
    int inner = ipow(N, d - 1 - axis);   /* stride of the axis */
    int outer = ipow(N, axis);
    long lines = (long)outer * inner;
#pragma omp parallel for schedule(static)
    for (long ln = 0; ln < lines; ++ln) {
        long o = ln / inner, in_ = ln % inner;
        long base = o * (long)N * inner + in_;
        for (int y = 0; y < N; ++y) {
            cplx acc = 0.0;
            const cplx *row = mat + (long)y * N;
            for (int x = 0; x < N; ++x) acc += row[x] * in[base + (long)x * inner];
            out[base + (long)y * inner] = acc;
        }
    }
}

/* f_hat_j = N^-d sum_x f(k_x) exp(-i pi j.k_x / L), j in [-N/2, N/2-1]^d
 * (eq. (fj) with the rectangle rule on the grid, which is exact for the
 * truncated series).  Output in FFT index order.  Pinned in the tests by the
 * round trip f_N(k_x) = f(k_x) and against numpy.fft with the (-1)^j grid
 * offset factor. */
int oracle_spectrum(int d, int N, double L, const double *f_in, double *fhat_out)
{
    if (d < 1 || d > 3 || N < 2 || (N & 1) || !f_in || !fhat_out) return ORACLE_ERR_INVALID;
    long n = ipow(N, d);
    double h = 2.0 * L / N;
    cplx *mat = malloc(sizeof(cplx) * N * N);
    cplx *a = malloc(sizeof(cplx) * n), *b = malloc(sizeof(cplx) * n);
    if (!mat || !a || !b) { free(mat); free(a); free(b); return ORACLE_ERR_NOMEM; }
    for (int i = 0; i < N; ++i)
        for (int x = 0; x < N; ++x) {
            double k = -L + h * x;
            mat[(long)i * N + x] = cexp(-I * M_PI * signed_mode(i, N) * k / L) / N;
        }
    memcpy(a, f_in, sizeof(cplx) * n);
    for (int ax = 0; ax < d; ++ax) {
        apply_axis(d, N, ax, mat, a, b);
        cplx *t = a; a = b; b = t;
    }
    memcpy(fhat_out, a, sizeof(cplx) * n);
    free(mat); free(a); free(b);
    return ORACLE_OK;
}

/* Evaluate the truncated series f_N(k) = sum_j f_hat_j exp(i pi j.k/L) at
 * the shifted grid k_x - s for a shift vector s (eq. (fj)).  Separable direct
 * sums, d passes of N^(d+1). */
static int eval_shifted(int d, int N, double L, const cplx *fhat, const double *s,
                        cplx *out, cplx *tmp, cplx *mat)
{
    long n = ipow(N, d);
    double h = 2.0 * L / N;
    const cplx *src = fhat;
    cplx *bufs[2] = {tmp, out};
    /* choose ping-pong so the last pass lands in `out` */
    int which = (d % 2 == 0) ? 0 : 1;
    for (int ax = 0; ax < d; ++ax) {
        for (int x = 0; x < N; ++x)
            for (int i = 0; i < N; ++i) {
                double k = -L + h * x - s[ax];
                mat[(long)x * N + i] = cexp(I * M_PI * signed_mode(i, N) * k / L);
            }
        cplx *dst = bufs[which];
        apply_axis(d, N, ax, mat, src, dst);
        src = dst;
        which ^= 1;
    }
    (void)n;
    return ORACLE_OK;
}

/* Inverse of oracle_spectrum: g(k_x) = sum_j ghat_j exp(i pi j.k_x/L). */
int oracle_synthesis(int d, int N, double L, const double *ghat, double *g_out)
{
    if (d < 1 || d > 3 || N < 2 || (N & 1) || !ghat || !g_out) return ORACLE_ERR_INVALID;
    long n = ipow(N, d);
    cplx *tmp = malloc(sizeof(cplx) * n), *mat = malloc(sizeof(cplx) * N * N);
    if (!tmp || !mat) { free(tmp); free(mat); return ORACLE_ERR_NOMEM; }
    double zero[3] = {0, 0, 0};
    eval_shifted(d, N, L, (const cplx *)ghat, zero, (cplx *)g_out, tmp, mat);
    free(tmp); free(mat);
    return ORACLE_OK;
}

/* f_N at arbitrary points k (npts x d, row-major), by the full d-dimensional
 * direct sum of eq. (fj).  Used for sampled-point checks. */
int oracle_eval_points(int d, int N, double L, const double *fhat_in, int npts,
                       const double *k, double *out)
{
    if (d < 1 || d > 3 || N < 2 || N > 512 || !fhat_in || !k || !out) return ORACLE_ERR_INVALID;
    const cplx *fhat = (const cplx *)fhat_in;
    long n = ipow(N, d);
#pragma omp parallel for schedule(static)
    for (int p = 0; p < npts; ++p) {
        cplx ph[3][512];
        for (int a = 0; a < d; ++a)
            for (int i = 0; i < N; ++i)
                ph[a][i] = cexp(I * M_PI * signed_mode(i, N) * k[p * d + a] / L);
        cplx acc = 0.0;
        for (long idx = 0; idx < n; ++idx) {
            long r = idx;
            cplx w = 1.0;
            for (int a = d - 1; a >= 0; --a) { w *= ph[a][r % N]; r /= N; }
            acc += w * fhat[idx];
        }
        ((cplx *)out)[p] = acc;
    }
    return ORACLE_OK;
}

/* ------------------------------------------------------------------------ */
/* The collision operator.                                                   */
/*                                                                           */
/* Nodes are passed explicitly: nr radial nodes r[] with weights wr[] (the   */
/* Gauss-Legendre rule mapped to [0, R]), ns directions qh[] (ns x d) with   */
/* weights ws[], nsig collision angles sg[] (nsig x d) with weights wsig[].  */
/* Triple p = (p1, p2, p3) carries W_p = wr r^(2d-3) ws wsig (eq. (G1): the  */
/* kernel |q|^(d-2) times the polar Jacobian |q|^(d-1)).                     */
/* Shifts: s_a = r qh, s_b = r (qh - sigma)/2, s_c = r (qh + sigma)/2; the    */
/* factors a, b, c of Alg. 1 are f_N(k - s_a) = f(k - q) = f(k_2),            */
/* f_N(k - s_b) = f(k') and f_N(k - s_c) = f(k'_2) (eq. (bkbk') with          */
/* k_2 = k - q).                                                              */
/* ------------------------------------------------------------------------ */

static void shift_vectors(int d, double r, const double *qh, const double *sg,
                          double *sa, double *sb, double *sc)
{
    for (int a = 0; a < d; ++a) {
        sa[a] = r * qh[a];
        sb[a] = 0.5 * r * (qh[a] - sg[a]);
        sc[a] = 0.5 * r * (qh[a] + sg[a]);
    }
}

/* Physical (grid) form of the operator: at every grid point,
 *   Q = 2^(1-d) sum_p W_p [ b a c - F0 a c + b F0 c - b a F0 ],
 * with F0 = f_N(k_x).  The four bracket terms are K_1..K_4 of eq.
 * (WKE-Boltz) with the sphere integral and the q integral replaced by the
 * quadrature of eq. (G1).  K_out (if non-NULL) receives the four sums
 * sum_p W_p [term] (without the 2^(1-d) factor), one N^d block each.
 * In exact arithmetic this equals the inverse transform of the cyclic
 * double-convolution form (oracle_Q_fourier); the tests pin the two
 * against each other. */
int oracle_Q_physical(int d, int N, double L,
                      int nr, const double *r, const double *wr,
                      int ns, const double *qh, const double *ws,
                      int nsig, const double *sg, const double *wsig,
                      const double *f_in, double *Q_out, double *K_out)
{
    if (d < 2 || d > 3 || N < 2 || (N & 1) || nr < 1 || ns < 1 || nsig < 1) return ORACLE_ERR_INVALID;
    if (!r || !wr || !qh || !ws || !sg || !wsig || !f_in || !Q_out) return ORACLE_ERR_INVALID;
    long n = ipow(N, d);
    cplx *fhat = malloc(sizeof(cplx) * n);
    cplx *F0 = malloc(sizeof(cplx) * n), *A = malloc(sizeof(cplx) * n);
    cplx *B = malloc(sizeof(cplx) * n), *C = malloc(sizeof(cplx) * n);
    cplx *tmp = malloc(sizeof(cplx) * n), *mat = malloc(sizeof(cplx) * N * N);
    cplx *K = calloc(4 * n, sizeof(cplx));
    if (!fhat || !F0 || !A || !B || !C || !tmp || !mat || !K) {
        free(fhat); free(F0); free(A); free(B); free(C); free(tmp); free(mat); free(K);
        return ORACLE_ERR_NOMEM;
    }
    oracle_spectrum(d, N, L, f_in, (double *)fhat);
    double zero[3] = {0, 0, 0};
    eval_shifted(d, N, L, fhat, zero, F0, tmp, mat);
    for (int p1 = 0; p1 < nr; ++p1) {
        double rr = r[p1];
        double radial = wr[p1] * pow(rr, 2 * d - 3);
        for (int p2 = 0; p2 < ns; ++p2) {
            double sa[3], sb[3], sc[3];
            shift_vectors(d, rr, qh + p2 * d, sg, sa, sb, sc);
            eval_shifted(d, N, L, fhat, sa, A, tmp, mat);
            for (int p3 = 0; p3 < nsig; ++p3) {
                double W = radial * ws[p2] * wsig[p3];
                shift_vectors(d, rr, qh + p2 * d, sg + p3 * d, sa, sb, sc);
                eval_shifted(d, N, L, fhat, sb, B, tmp, mat);
                eval_shifted(d, N, L, fhat, sc, C, tmp, mat);
#pragma omp parallel for schedule(static)
                for (long x = 0; x < n; ++x) {
                    K[x]         += W * (B[x] * A[x] * C[x]);
                    K[n + x]     += W * (F0[x] * A[x] * C[x]);
                    K[2 * n + x] += W * (B[x] * F0[x] * C[x]);
                    K[3 * n + x] += W * (B[x] * A[x] * F0[x]);
                }
            }
        }
    }
    double pref = ldexp(1.0, 1 - d);
    cplx *Q = (cplx *)Q_out;
    for (long x = 0; x < n; ++x) Q[x] = pref * (K[x] - K[n + x] + K[2 * n + x] - K[3 * n + x]);
    if (K_out) memcpy(K_out, K, sizeof(cplx) * 4 * n);
    free(fhat); free(F0); free(A); free(B); free(C); free(tmp); free(mat); free(K);
    return ORACLE_OK;
}

/* Physical form at selected grid points only (flat indices idx[]), with each
 * shifted value f_N(k_x - s) computed by the full d-dimensional direct sum.
 * Cost M * 3 * N^d per point; used to check full-size GPU outputs. */
int oracle_Q_points(int d, int N, double L,
                    int nr, const double *r, const double *wr,
                    int ns, const double *qh, const double *ws,
                    int nsig, const double *sg, const double *wsig,
                    const double *f_in, int npts, const long *idx, double *Q_out)
{
    if (d < 2 || d > 3 || N < 2 || (N & 1) || !f_in || !idx || !Q_out) return ORACLE_ERR_INVALID;
    long n = ipow(N, d);
    double h = 2.0 * L / N;
    cplx *fhat = malloc(sizeof(cplx) * n);
    if (!fhat) return ORACLE_ERR_NOMEM;
    oracle_spectrum(d, N, L, f_in, (double *)fhat);
    int ntr = nr * ns * nsig;
    /* for each point, the shifted evaluation points: a per (p1,p2), b,c per triple */
    for (int p = 0; p < npts; ++p) {
        double kx[3];
        long rem = idx[p];
        for (int a = d - 1; a >= 0; --a) { kx[a] = -L + h * (rem % N); rem /= N; }
        int nq = 1 + nr * ns + 2 * ntr;
        double *pts = malloc(sizeof(double) * d * nq);
        cplx *val = malloc(sizeof(cplx) * nq);
        if (!pts || !val) { free(pts); free(val); free(fhat); return ORACLE_ERR_NOMEM; }
        for (int a = 0; a < d; ++a) pts[a] = kx[a];
        int q = 1;
        for (int p1 = 0; p1 < nr; ++p1)
            for (int p2 = 0; p2 < ns; ++p2) {
                double sa[3], sb[3], sc[3];
                shift_vectors(d, r[p1], qh + p2 * d, sg, sa, sb, sc);
                for (int a = 0; a < d; ++a) pts[q * d + a] = kx[a] - sa[a];
                ++q;
            }
        for (int p1 = 0; p1 < nr; ++p1)
            for (int p2 = 0; p2 < ns; ++p2)
                for (int p3 = 0; p3 < nsig; ++p3) {
                    double sa[3], sb[3], sc[3];
                    shift_vectors(d, r[p1], qh + p2 * d, sg + p3 * d, sa, sb, sc);
                    for (int a = 0; a < d; ++a) pts[q * d + a] = kx[a] - sb[a];
                    ++q;
                    for (int a = 0; a < d; ++a) pts[q * d + a] = kx[a] - sc[a];
                    ++q;
                }
        oracle_eval_points(d, N, L, (double *)fhat, nq, pts, (double *)val);
        cplx F0 = val[0], acc = 0.0;
        int qa = 1, qb = 1 + nr * ns;
        for (int p1 = 0; p1 < nr; ++p1) {
            double radial = wr[p1] * pow(r[p1], 2 * d - 3);
            for (int p2 = 0; p2 < ns; ++p2) {
                cplx A = val[qa++];
                for (int p3 = 0; p3 < nsig; ++p3) {
                    cplx B = val[qb++], C = val[qb++];
                    double W = radial * ws[p2] * wsig[p3];
                    acc += W * (B * A * C - F0 * A * C + B * F0 * C - B * A * F0);
                }
            }
        }
        ((cplx *)Q_out)[p] = ldexp(1.0, 1 - d) * acc;
        free(pts); free(val);
    }
    free(fhat);
    return ORACLE_OK;
}

/* ------------------------------------------------------------------------ */
/* Fourier form: the double convolution of eq. (K1_con) and its K_2..K_4     */
/* analogues, summed directly.                                               */
/* ------------------------------------------------------------------------ */

/* Index helpers for a box of side `side` whose first slot is mode `lo`.   */
typedef struct { int d, side, lo; } box_t;

static long box_index(const box_t *b, const int *j)
{
    long idx = 0;
    for (int a = 0; a < b->d; ++a) {
        int u = j[a] - b->lo;
        if (u < 0 || u >= b->side) return -1;
        idx = idx * b->side + u;
    }
    return idx;
}

static void box_modes(const box_t *b, long idx, int *j)
{
    for (int a = b->d - 1; a >= 0; --a) { j[a] = (int)(idx % b->side) + b->lo; idx /= b->side; }
}

/* wrap a signed mode into [-N/2, N/2-1] */
static int wrap_mode(int j, int N)
{
    int u = ((j + N / 2) % N + N) % N;
    return u - N / 2;
}

/* FFT-order slot of a signed mode in [-N/2, N/2-1] */
static int slot_of(int j, int N) { return j >= 0 ? j : j + N; }

static long fft_index(int d, int N, const int *j)
{
    long idx = 0;
    for (int a = 0; a < d; ++a) idx = idx * N + slot_of(j[a], N);
    return idx;
}

/* Convolution inner sum: out(u) = sum_{l in J} X_l Y_{u-l}, for u in the
 * output box.  In cyclic mode u - l wraps into J (size-N transforms, Alg. 1);
 * in linear mode terms with u - l outside J are dropped (the exact
 * constraint l + n = j - m of eq. (KK1)).  X, Y are in FFT order. */
static void conv_inner(int d, int N, int linear, const cplx *X, const cplx *Y,
                       const box_t *ob, cplx *out)
{
    long nout = ipow(ob->side, d);
    long n = ipow(N, d);
#pragma omp parallel for schedule(static)
    for (long o = 0; o < nout; ++o) {
        int u[3], l[3], v[3];
        box_modes(ob, o, u);
        cplx acc = 0.0;
        for (long li = 0; li < n; ++li) {
            long rem = li;
            for (int a = d - 1; a >= 0; --a) { l[a] = signed_mode((int)(rem % N), N); rem /= N; }
            int ok = 1;
            for (int a = 0; a < d; ++a) {
                v[a] = u[a] - l[a];
                if (linear) { if (v[a] < -N / 2 || v[a] > N / 2 - 1) { ok = 0; break; } }
                else v[a] = wrap_mode(v[a], N);
            }
            if (!ok) continue;
            acc += X[li] * Y[fft_index(d, N, v)];
        }
        out[o] = acc;
    }
}

/* Outer sum: out_j = sum_{m in J} Z_m F(j - m) for j in J, with F given on
 * box ib (cyclic: j - m wraps; linear: j - m is always inside ib). */
static void conv_outer(int d, int N, int linear, const cplx *Z, const cplx *F,
                       const box_t *ib, cplx *out)
{
    long n = ipow(N, d);
#pragma omp parallel for schedule(static)
    for (long ji = 0; ji < n; ++ji) {
        int j[3], m[3], u[3];
        long rem = ji;
        for (int a = d - 1; a >= 0; --a) { j[a] = signed_mode((int)(rem % N), N); rem /= N; }
        cplx acc = 0.0;
        for (long mi = 0; mi < n; ++mi) {
            long r2 = mi;
            for (int a = d - 1; a >= 0; --a) { m[a] = signed_mode((int)(r2 % N), N); r2 /= N; }
            for (int a = 0; a < d; ++a) {
                u[a] = j[a] - m[a];
                if (!linear) u[a] = wrap_mode(u[a], N);
            }
            long fi = box_index(ib, u);
            if (fi >= 0) acc += Z[mi] * F[fi];
        }
        out[ji] = acc;
    }
}

/* Fourier form of the operator (eqs. (K1_con) and the K_2..K_4 analogues):
 *   K_hat_1 = sum_p W_p sum_m A_m F_1(j-m),  F_1 = B (*) C
 *   K_hat_2 = sum_p W_p sum_m A_m F_2(j-m),  F_2 = F (*) C
 *   K_hat_3 = sum_p W_p sum_m F_m F_3(j-m),  F_3 = B (*) C
 *   K_hat_4 = sum_p W_p sum_m A_m F_4(j-m),  F_4 = B (*) F
 * with F = f_hat, A = alpha f_hat = exp(-i pi j.s_a/L) f_hat,
 * B = beta beta~ f_hat = exp(-i pi j.s_b/L) f_hat and
 * C = gamma gamma~ f_hat = exp(-i pi j.s_c/L) f_hat (eq. (G1) phase factors;
 * the gamma~ factor uses sigma as in eq. (G1)).
 * Q_hat = 2^(1-d) (K_hat_1 - K_hat_2 + K_hat_3 - K_hat_4) (Alg. 1 combine),
 * returned on the grid by the direct inverse sum.  Khat_out (optional)
 * receives the four K_hat_l (no 2^(1-d)) in FFT order; Qhat_out (optional)
 * receives Q_hat.  Cost 7 N^(2d) complex products per triple (cyclic). */
int oracle_Q_fourier(int d, int N, double L,
                     int nr, const double *r, const double *wr,
                     int ns, const double *qh, const double *ws,
                     int nsig, const double *sg, const double *wsig,
                     int linear, const double *f_in, double *Q_out,
                     double *Qhat_out, double *Khat_out)
{
    if (d < 2 || d > 3 || N < 2 || (N & 1) || nr < 1 || ns < 1 || nsig < 1) return ORACLE_ERR_INVALID;
    if (!r || !wr || !qh || !ws || !sg || !wsig || !f_in || !Q_out) return ORACLE_ERR_INVALID;
    long n = ipow(N, d);
    box_t ib;
    ib.d = d;
    if (linear) { ib.side = 2 * N - 1; ib.lo = -N + 1; }   /* j - m in [-N+1, N-1] */
    else { ib.side = N; ib.lo = -N / 2; }
    long ni = ipow(ib.side, d);
    cplx *F = malloc(sizeof(cplx) * n), *A = malloc(sizeof(cplx) * n);
    cplx *B = malloc(sizeof(cplx) * n), *C = malloc(sizeof(cplx) * n);
    cplx *in1 = malloc(sizeof(cplx) * ni), *in2 = malloc(sizeof(cplx) * ni), *in4 = malloc(sizeof(cplx) * ni);
    cplx *o = malloc(sizeof(cplx) * n);
    cplx *Kh = calloc(4 * n, sizeof(cplx));
    cplx *Qh = malloc(sizeof(cplx) * n);
    if (!F || !A || !B || !C || !in1 || !in2 || !in4 || !o || !Kh || !Qh) {
        free(F); free(A); free(B); free(C); free(in1); free(in2); free(in4); free(o); free(Kh); free(Qh);
        return ORACLE_ERR_NOMEM;
    }
    oracle_spectrum(d, N, L, f_in, (double *)F);
    for (int p1 = 0; p1 < nr; ++p1) {
        double rr = r[p1];
        double radial = wr[p1] * pow(rr, 2 * d - 3);
        for (int p2 = 0; p2 < ns; ++p2)
            for (int p3 = 0; p3 < nsig; ++p3) {
                double sa[3], sb[3], sc[3];
                shift_vectors(d, rr, qh + p2 * d, sg + p3 * d, sa, sb, sc);
                double W = radial * ws[p2] * wsig[p3];
                for (long ji = 0; ji < n; ++ji) {
                    int j[3];
                    long rem = ji;
                    for (int a = d - 1; a >= 0; --a) { j[a] = signed_mode((int)(rem % N), N); rem /= N; }
                    double pa = 0, pb = 0, pc = 0;
                    for (int a = 0; a < d; ++a) { pa += j[a] * sa[a]; pb += j[a] * sb[a]; pc += j[a] * sc[a]; }
                    A[ji] = cexp(-I * M_PI * pa / L) * F[ji];
                    B[ji] = cexp(-I * M_PI * pb / L) * F[ji];
                    C[ji] = cexp(-I * M_PI * pc / L) * F[ji];
                }
                conv_inner(d, N, linear, B, C, &ib, in1);   /* F_1 = F_3 */
                conv_inner(d, N, linear, F, C, &ib, in2);   /* F_2 */
                conv_inner(d, N, linear, B, F, &ib, in4);   /* F_4 */
                conv_outer(d, N, linear, A, in1, &ib, o);
                for (long x = 0; x < n; ++x) Kh[x] += W * o[x];
                conv_outer(d, N, linear, A, in2, &ib, o);
                for (long x = 0; x < n; ++x) Kh[n + x] += W * o[x];
                conv_outer(d, N, linear, F, in1, &ib, o);
                for (long x = 0; x < n; ++x) Kh[2 * n + x] += W * o[x];
                conv_outer(d, N, linear, A, in4, &ib, o);
                for (long x = 0; x < n; ++x) Kh[3 * n + x] += W * o[x];
            }
    }
    double pref = ldexp(1.0, 1 - d);
    for (long x = 0; x < n; ++x) Qh[x] = pref * (Kh[x] - Kh[n + x] + Kh[2 * n + x] - Kh[3 * n + x]);
    oracle_synthesis(d, N, L, (const double *)Qh, Q_out);
    if (Qhat_out) memcpy(Qhat_out, Qh, sizeof(cplx) * n);
    if (Khat_out) memcpy(Khat_out, Kh, sizeof(cplx) * 4 * n);
    free(F); free(A); free(B); free(C); free(in1); free(in2); free(in4); free(o); free(Kh); free(Qh);
    return ORACLE_OK;
}

/* ------------------------------------------------------------------------ */
/* Time stepping and moments.                                                */
/* ------------------------------------------------------------------------ */

/* Classical fourth-order Runge-Kutta (the paper's RK4; the variant is not
 * stated, the classical one is used) on the grid state f, with Q from the
 * physical form.  f is updated in place, nsteps steps of size dt. */
int oracle_rk4(int d, int N, double L,
               int nr, const double *r, const double *wr,
               int ns, const double *qh, const double *ws,
               int nsig, const double *sg, const double *wsig,
               double *f_io, double dt, int nsteps)
{
    if (d < 2 || d > 3 || !f_io || nsteps < 0) return ORACLE_ERR_INVALID;
    long n = ipow(N, d);
    cplx *y = (cplx *)f_io;
    cplx *k = malloc(sizeof(cplx) * n), *ys = malloc(sizeof(cplx) * n), *acc = malloc(sizeof(cplx) * n);
    if (!k || !ys || !acc) { free(k); free(ys); free(acc); return ORACLE_ERR_NOMEM; }
    static const double cstage[4] = {0.0, 0.5, 0.5, 1.0};
    static const double bweight[4] = {1.0, 2.0, 2.0, 1.0};
    for (int st = 0; st < nsteps; ++st) {
        for (long x = 0; x < n; ++x) acc[x] = 0.0;
        for (int s = 0; s < 4; ++s) {
            if (s == 0) memcpy(ys, y, sizeof(cplx) * n);
            else for (long x = 0; x < n; ++x) ys[x] = y[x] + cstage[s] * dt * k[x];
            int rc = oracle_Q_physical(d, N, L, nr, r, wr, ns, qh, ws, nsig, sg, wsig,
                                       (const double *)ys, (double *)k, NULL);
            if (rc) { free(k); free(ys); free(acc); return rc; }
            for (long x = 0; x < n; ++x) acc[x] += bweight[s] * k[x];
        }
        for (long x = 0; x < n; ++x) y[x] += dt / 6.0 * acc[x];
    }
    free(k); free(ys); free(acc);
    return ORACLE_OK;
}

/* Moments by the rectangle rule on the grid (the paper's rho and E):
 * out = [rho, E, P_1..P_d, max|Im f|] with rho = h^d sum Re f,
 * E = h^d sum Re f |k_x|^2 and P_a = h^d sum Re f k_a. */
int oracle_moments(int d, int N, double L, const double *f_in, double *out)
{
    if (d < 1 || d > 3 || !f_in || !out) return ORACLE_ERR_INVALID;
    long n = ipow(N, d);
    double h = 2.0 * L / N, hd = pow(h, d);
    double rho = 0, E = 0, P[3] = {0, 0, 0}, mim = 0;
    const cplx *f = (const cplx *)f_in;
    for (long x = 0; x < n; ++x) {
        double k[3], k2 = 0;
        long rem = x;
        for (int a = d - 1; a >= 0; --a) { k[a] = -L + h * (rem % N); rem /= N; k2 += k[a] * k[a]; }
        double fr = creal(f[x]);
        rho += fr;
        E += fr * k2;
        for (int a = 0; a < d; ++a) P[a] += fr * k[a];
        double ai = fabs(cimag(f[x]));
        if (ai > mim) mim = ai;
    }
    out[0] = hd * rho;
    out[1] = hd * E;
    for (int a = 0; a < d; ++a) out[2 + a] = hd * P[a];
    out[2 + d] = mim;
    return ORACLE_OK;
}

/* ------------------------------------------------------------------------ */
/* Exact-weight reference system (Appendix B).                               */
/* ------------------------------------------------------------------------ */

/* Integral of e^{i x.s} over the unit sphere S^{d-1}, |x| = x: 2 pi J_0(x)
 * in 2D, 4 pi sin(x)/x in 3D. */
static double sphere_mean(int d, double x)
{
    if (d == 2) return 2.0 * M_PI * j0(x);
    return x == 0.0 ? 4.0 * M_PI : 4.0 * M_PI * sin(x) / x;
}

/* The Galerkin system of eqs. (KK1)-(KK4) without the fast algorithm: the
 * exact constraint l + m + n = j (Appendix B) and the weight functions
 * G_1..G_4 with their q-hat and sigma integrals in closed form.  Each G is
 * an integral over |q| = r in [0, R] of r^{2d-3} times two sphere means:
 *   G_1(l,m,n) = Phi(|2m+l+n|^2, |l-n|^2),  G_2(m,n) = Phi(|2m+n|^2, |n|^2),
 *   G_3(l,n)   = Phi(|l+n|^2, |l-n|^2),     G_4(l,m) = Phi(|2m+l|^2, |l|^2),
 *   Phi(a, b)  = int_0^R r^{2d-3} S(pi r sqrt(a) / (2L)) S(pi r sqrt(b) / (2L)) dr,
 * S the sphere mean above; the r integral by nr-point Gauss-Legendre.  Then
 *   Q_hat_j = 2^{1-d} sum_{l,m,n in J, l+m+n=j} (G_1 - G_2 + G_3 - G_4) f_l f_m f_n
 * and Q on the grid by the direct inverse transform.  O(N^{3d}): tiny N.
 * Parity pinned by the tests: zero mass mode (Appendix B), and the fast
 * method with the exact constraint converges to it as its quadrature is
 * refined. */
int oracle_exact_system(int d, int N, double L, double R, int nr, const double *f_in, double *Q_out,
                        double *Qhat_out)
{
    if (d < 2 || d > 3 || N < 2 || (N & 1) || nr < 1 || !f_in || !Q_out || !(L > 0) || !(R > 0))
        return ORACLE_ERR_INVALID;
    long n = ipow(N, d);
    const int A = 4 * d * N * N, B = d * (N - 1) * (N - 1);
    double *t = malloc(sizeof(double) * nr), *w = malloc(sizeof(double) * nr);
    double *Sa = malloc(sizeof(double) * (size_t)(A + 1) * nr);
    double *phi = malloc(sizeof(double) * (size_t)(A + 1) * (B + 1));
    cplx *F = malloc(sizeof(cplx) * n), *Qh = malloc(sizeof(cplx) * n);
    if (!t || !w || !Sa || !phi || !F || !Qh) {
        free(t); free(w); free(Sa); free(phi); free(F); free(Qh);
        return ORACLE_ERR_NOMEM;
    }
    oracle_gauss_legendre(nr, t, w);
    for (int a = 0; a <= A; ++a)
        for (int k = 0; k < nr; ++k) {
            const double r = 0.5 * R * (1.0 + t[k]);
            Sa[(size_t)a * nr + k] = sphere_mean(d, M_PI * r * sqrt((double)a) / (2.0 * L));
        }
#pragma omp parallel for schedule(static)
    for (int a = 0; a <= A; ++a)
        for (int b = 0; b <= B; ++b) {
            double acc = 0.0;
            for (int k = 0; k < nr; ++k) {
                const double r = 0.5 * R * (1.0 + t[k]);
                acc += 0.5 * R * w[k] * pow(r, 2 * d - 3) * Sa[(size_t)a * nr + k] * Sa[(size_t)b * nr + k];
            }
            phi[(size_t)a * (B + 1) + b] = acc;
        }
    oracle_spectrum(d, N, L, f_in, (double *)F);
#pragma omp parallel for schedule(static)
    for (long ji = 0; ji < n; ++ji) {
        int j[3] = {0, 0, 0}, l[3] = {0, 0, 0}, m[3] = {0, 0, 0}, v[3] = {0, 0, 0};
        long rem = ji;
        for (int a = d - 1; a >= 0; --a) { j[a] = signed_mode((int)(rem % N), N); rem /= N; }
        cplx acc = 0.0;
        for (long li = 0; li < n; ++li) {
            long r1 = li;
            for (int a = d - 1; a >= 0; --a) { l[a] = signed_mode((int)(r1 % N), N); r1 /= N; }
            for (long mi = 0; mi < n; ++mi) {
                long r2 = mi;
                for (int a = d - 1; a >= 0; --a) { m[a] = signed_mode((int)(r2 % N), N); r2 /= N; }
                int ok = 1;
                for (int a = 0; a < d; ++a) {
                    v[a] = j[a] - l[a] - m[a];
                    if (v[a] < -N / 2 || v[a] > N / 2 - 1) ok = 0;
                }
                if (!ok) continue;
                int q1 = 0, q2 = 0, q3 = 0, q4 = 0, q5 = 0, q6 = 0, q7 = 0, q8 = 0;
                for (int a = 0; a < d; ++a) {
                    const int u1 = 2 * m[a] + l[a] + v[a], u2 = l[a] - v[a], u3 = 2 * m[a] + v[a];
                    const int u4 = l[a] + v[a], u5 = 2 * m[a] + l[a];
                    q1 += u1 * u1; q2 += u2 * u2; q3 += u3 * u3; q4 += v[a] * v[a];
                    q5 += u4 * u4; q6 += u2 * u2; q7 += u5 * u5; q8 += l[a] * l[a];
                }
                const double G = phi[(size_t)q1 * (B + 1) + q2] - phi[(size_t)q3 * (B + 1) + q4]
                               + phi[(size_t)q5 * (B + 1) + q6] - phi[(size_t)q7 * (B + 1) + q8];
                acc += G * F[li] * F[mi] * F[fft_index(d, N, v)];
            }
        }
        Qh[ji] = ldexp(1.0, 1 - d) * acc;
    }
    if (Qhat_out) memcpy(Qhat_out, Qh, sizeof(cplx) * n);
    oracle_synthesis(d, N, L, (const double *)Qh, Q_out);
    free(t); free(w); free(Sa); free(phi); free(F); free(Qh);
    return ORACLE_OK;
}

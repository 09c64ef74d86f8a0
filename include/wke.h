/*
 * wke.h -- C interface of the MI355X (gfx950) library for the spectrally
 * truncated four-wave collision operator Q(f) = K^R(f,f,f) and its explicit
 * time integration, after Qi, Shen and Wang, "A fast Fourier spectral method
 * for wave kinetic equation" (arXiv 2503.12805).
 *
 * What is computed (paper references by section / equation / algorithm):
 *   - f is the wave action density sampled on the uniform grid of the box
 *     D_L = [-L, L]^d (Section 3.2, Step 1): node x in {0..N-1} per axis sits
 *     at k = -L + h x, h = 2L/N.  Its truncated Fourier series f_N keeps the
 *     modes j in [-N/2, N/2-1]^d (eq. (fj)), so f_N is complex off the grid:
 *     all grid data are complex.
 *   - Q = 2^(1-d) [K_1 - K_2 + K_3 - K_4] (eq. (WKE-Boltz) and the final
 *     combine of Alg. 1) with the integrals over |q| in [0, R], q-hat and
 *     sigma replaced by Gauss-Legendre, midpoint (2D) or spherical-design (3D)
 *     rules (eq. (G1)), and every discrete convolution of Alg. 1 taken with
 *     size-N transforms, i.e. cyclic in the mode index.  The result is
 *     returned on the grid (the last step of Alg. 1).
 *   - wke_step advances df/dt = Q(f) with classical RK4 (Sections 4.1.2 and
 *     4.2.2 use "RK4").
 *   - wke_moments returns the mass and energy of Section 2 (and momentum) by
 *     the rectangle rule on the grid.
 *
 * Memory: every array argument marked "device" is GPU memory allocated and
 * owned by the caller (for example a torch tensor); the library never frees
 * or keeps it past the call.  Grid arrays are complex128 interleaved
 * (re, im), row-major with the last axis fastest, and the instances of a
 * batch are packed back to back: instance i starts at complex element
 * wke_offset(plan, i) and has N_i^d elements; wke_total_elems(plan) is the
 * packed length.  A plan owns its quadrature tables and workspace.
 *
 * Streams: every call is enqueued on the plan's stream and returns without
 * waiting, except wke_moments and wke_get_nodes, which wait for their
 * results.  One plan must not be used from two host threads at once, and
 * calls on one plan must not overlap on different streams.
 *
 * Errors: functions return a wke_status; nothing throws across this
 * interface.  wke_last_error() gives a message for the calling thread's
 * last failure.
 */
#ifndef WKE_H
#define WKE_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct wke_plan_s *wke_plan_t;

typedef enum {
    WKE_OK = 0,
    WKE_ERR_INVALID = -1,      /* bad argument or descriptor */
    WKE_ERR_UNSUPPORTED = -2,  /* valid but not built (grid size, rule) */
    WKE_ERR_HIP = -3,          /* a HIP runtime call failed */
    WKE_ERR_NOMEM = -4,        /* device allocation failed */
    WKE_ERR_NONFINITE = -5     /* a moment came out NaN or infinite */
} wke_status;

/* Sphere rules (eq. (G1)); the same rule is used for q-hat and sigma. */
enum {
    WKE_MIDPOINT = 0,     /* 2D: angles (2i+1) pi / n, weights 2 pi / n      */
    WKE_OCTAHEDRON = 1,   /* 3D: 6 points +-e_a, weights 4 pi / 6            */
    WKE_CUBE = 2,         /* 3D: 8 points (+-1,+-1,+-1)/sqrt 3               */
    WKE_ICOSAHEDRON = 3   /* 3D: 12 vertices (0,+-1,+-phi)/sqrt(1+phi^2), cyclic */
};

/* Arithmetic of the transforms and products. */
enum {
    WKE_F64 = 0,          /* everything in double                            */
    WKE_F32 = 1           /* transforms and products in float; quadrature
                             tables built in double and rounded once; the
                             sum over quadrature points compensated
                             (Neumaier); state, time-stepping, cross-block
                             sums and moments in double                       */
};

/* One problem instance. */
typedef struct {
    int d;            /* dimension, 2 or 3                                    */
    int N;            /* modes per axis: 2D 16, 32, 48, 64, 96, 128;
                         3D 16, 32, 64                                        */
    double L;         /* half-width of the periodic box D_L = [-L, L]^d       */
    double R;         /* radius of the |q| integral; <= 0 selects
                         R = 4L/(3+sqrt 2), the equality case of the
                         anti-aliasing condition L >= (3+sqrt 2) S / 2 with
                         R = 2S (Section 3.2, Step 1)                         */
    int N_r;          /* Gauss-Legendre points in |q| (>= 1)                  */
    int N_s;          /* points of the q-hat rule                             */
    int N_sig;        /* points of the sigma rule                             */
    int sphere_rule;  /* WKE_MIDPOINT (d = 2) or a 3D design (d = 3; N_s and
                         N_sig must equal its point count)                    */
} wke_desc;

/* Build a plan for `batch` instances (all of one dimension d).  precision is
 * WKE_F64 or WKE_F32; stream is a hipStream_t (NULL: the default stream).
 * The quadrature nodes, weights and phase tables are computed on the GPU in
 * double precision.  On success *out receives the plan. */
wke_status wke_plan_create(wke_plan_t *out, const wke_desc *insts, int batch, int precision,
                           void *stream);

/* The exact-weight reference system (Appendix B): the Galerkin sums of eqs.
 * (KK1)-(KK4) with the exact constraint l + m + n = j and the weight
 * functions G_1..G_4 integrated in closed form over q-hat and sigma (the
 * sphere mean of e^{i x.s} is 2 pi J_0(|x|) in 2D, 4 pi sin|x|/|x| in 3D),
 * over |q| in [0, R] by n_radial-point Gauss-Legendre.  Its zeroth mode
 * vanishes (mass is conserved).  It costs O(N^(3d)) and serves only to
 * measure the quadrature error of the fast method at tiny N: N^d <= 1024.
 * desc gives d, N, L and R (<= 0: 4L/(3+sqrt 2)); its quadrature counts and
 * rule are not used.  f: device, complex128 grid (N^d, read); Q: device,
 * same layout (written, may not alias f).  Allocates and frees its own
 * workspace (about 8 (4dN^2+1)(d(N-1)^2+1) bytes for the weight table) and
 * waits for completion on `stream`. */
wke_status wke_exact_system(const wke_desc *desc, int n_radial, const double *f, double *Q, void *stream);

/* The same reference system for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): no allocation, no free and no wait.  Its workspace (radial
 * nodes, sphere-mean and weight tables, spectra) lives in a static device
 * array of 16 MiB per GPU, held from the first call on that GPU until the
 * process ends.  Arguments and result as for wke_exact_system; the call is
 * enqueued on `stream` and returns without waiting.  Sizes whose workspace
 * exceeds the array are refused with WKE_ERR_UNSUPPORTED before any launch:
 * 8 (2 nr + (4dN^2+1)(nr + d(N-1)^2 + 1) + 4 N^d) bytes, rounded up per
 * table, must stay within 16 MiB (2D N = 16 with up to 256 radial points
 * fits; 2D N = 32 does not).  Every call on one GPU uses the same array:
 * calls that overlap on one GPU (on different streams, or from several host
 * threads) race and give wrong results; calls in order on one stream are
 * safe.  Nothing in the array needs to start at zero. */
wke_status wke_exact_system_noalloc(const wke_desc *desc, int n_radial, const double *f, double *Q, void *stream);

/* Build a plan for the Nyquist-zero real form: the operator applied to
 * Re f with every mode that has a component j_a = -N/2 dropped, i.e.
 * Q(P f) with P that projection.  Every mode of P f has its partner -j in the
 * box, so for real data every shifted field f_N(k - s) and every product is
 * real (the truncated series of eq. (fj) keeps j = -N/2 without its partner,
 * which is what makes f_N complex off the grid).  The column pass then
 * carries two real fields per complex transform and multiplies in real
 * arithmetic; the unshifted factor comes from a zero-shift field so that it
 * too is P f.  Q is returned on the grid with a zero imaginary part; wke_step
 * evolves Re f and leaves Im f unchanged.  Packing, offsets and every call
 * are as for wke_plan_create, except that the item-slot column pass does not
 * exist for this form (wke_plan_set_column_kernel(WKE_COLUMN_SLOTS) returns
 * WKE_ERR_UNSUPPORTED, as does a quadrature whose items do not fit the
 * field-parallel pass). */
wke_status wke_plan_create_real(wke_plan_t *out, const wke_desc *insts, int batch, int precision, void *stream);

/* Build an exact-Galerkin (de-aliased) plan: the same operator with the mode
 * constraint l + m + n = j of eq. (KK1) kept exactly, instead of modulo N,
 * as the remark on zero padding after the truncation in Section 3 suggests.
 * Grids, packing, offsets and every call taking a plan are as for
 * wke_plan_create; the difference is internal: the operator runs on the
 * grid of 2N points per axis (every shifted field is f_N sampled there), and
 * its result is projected back onto the modes [-N/2, N/2-1] on the grid of
 * N points.  A product of three fields with modes in [-N/2, N/2-1] has
 * modes in [-3N/2, 3N/2-3], none of which wraps into [-N/2, N/2-1] modulo
 * 2N, so 2N points suffice.  Needs 2N to be a built size: 2D N = 8, 16,
 * 24, 32, 48, 64; 3D N = 8, 16, 32 (WKE_ERR_UNSUPPORTED otherwise).  Graph
 * replay (wke_set_graphs) is not built for these plans.  wke_plan_tune,
 * wke_time_kernels, wke_plan_set_split, wke_plan_set_column_kernel,
 * wke_field_counts and wke_work_model act on (and report) the operator on
 * the grid of 2N points; wke_time_kernels and wke_plan_tune take the coarse
 * f and resample it first. */
wke_status wke_plan_create_galerkin(wke_plan_t *out, const wke_desc *insts, int batch, int precision,
                                    void *stream);

/* Release the plan and its device memory (waits for its stream). */
void wke_plan_destroy(wke_plan_t plan);

/* Complex-element offset of instance i in packed grid arrays, and the total
 * packed length (complex elements).  Return 0 / 0 for invalid arguments. */
size_t wke_offset(wke_plan_t plan, int instance);
size_t wke_total_elems(wke_plan_t plan);

/* Q = K^R(f, f, f) on the grid for every instance (Alg. 1).
 * f: device, complex128 packed grid (read only); Q: device, same layout
 * (written; may not alias f). */
wke_status wke_eval_Q(wke_plan_t plan, const double *f, double *Q);

/* Q_hat, the Fourier coefficients of Q in the series of eq. (fj):
 * Q_hat_j = N^-d sum_x Q(k_x) e^{-i pi j.k_x / L}, j in [-N/2, N/2-1]^d in
 * FFT index order (index i is mode i for i < N/2, else i - N), the form in
 * which Section 3 writes the Galerkin terms.  wke_eval_Q into Qhat, then one
 * in-place forward transform per axis in double.  f, Qhat: device,
 * complex128 packed, as for wke_eval_Q (Qhat may not alias f).
 * WKE_ERR_UNSUPPORTED, before any launch, for N outside 8, 16, 32, 48, 64,
 * 96, 128. */
wke_status wke_eval_Q_hat(wke_plan_t plan, const double *f, double *Qhat);

/* nsteps classical RK4 steps of size dt for df/dt = Q(f), in place.
 * f: device, complex128 packed grid (read and written).  Kernels are
 * launched directly on the plan's stream unless graph replay is switched on
 * (wke_set_graphs); results are bitwise the same either way. */
wke_status wke_step(wke_plan_t plan, double *f, double dt, int nsteps);

/* Switch graph replay of wke_step on (enable != 0) or off (the default).
 * When on, one step's kernel launches (a slab and a column pass per RK4
 * stage and N group) are captured once into a HIP graph (on a private
 * stream of the plan, keyed on f and dt) and replayed on the plan's stream
 * for every step; the groups of a concurrent plan are parallel branches of
 * that graph. */
wke_status wke_set_graphs(wke_plan_t plan, int enable);

/* Instances of different N form groups, each with its own launches (the
 * kernels are specialised on N).  The groups share no data, so a plan with
 * more than one group runs each group on a stream of its own
 * (concurrency on, the default for such plans): wke_eval_Q and wke_step
 * record an event on the plan's stream that every group stream waits for,
 * enqueue each group's launches on its stream, and make the plan's stream
 * wait for every group's last launch, so the call is ordered with other
 * work on the plan's stream as before.  The group streams are created on
 * first use at the default priority and destroyed with the plan.
 * enable = 0 puts every launch on the plan's stream, one group after the
 * other.  Results are bitwise the same either way.  Exact-Galerkin plans
 * always run their groups in order. */
wke_status wke_plan_set_concurrency(wke_plan_t plan, int enable);

/* Number of N groups of the plan (distinct N among its instances; 0 for a
 * NULL plan). */
int wke_plan_groups(wke_plan_t plan);

/* Moments of every instance by the rectangle rule on the grid, waiting for
 * the result: out is host memory of 6 * batch doubles, per instance
 * [rho, E, P_1, P_2, P_3, max|Im f|] with rho = h^d sum Re f,
 * E = h^d sum Re f |k|^2, P_a = h^d sum Re f k_a (P_3 = 0 when d = 2).
 * f: device, complex128 packed grid.  Returns WKE_ERR_NONFINITE (with out
 * filled) if any value is NaN or infinite. */
wke_status wke_moments(wke_plan_t plan, const double *f, double *out);

/* Copy the quadrature of instance i, as built on the GPU, to host arrays:
 * r[N_r], wr[N_r] (radial nodes on [0, R] and weights), qh[N_s*d], ws[N_s],
 * sg[N_sig*d], wsig[N_sig].  Waits for the copy. */
wke_status wke_get_nodes(wke_plan_t plan, int instance, double *r, double *wr, double *qh,
                         double *ws, double *sg, double *wsig);

/* Autotune the plan on the input f (device, packed grid; Q is written as
 * scratch; the plan's RK4 stage buffers too): for every group of
 * instances that share N, time the slab pass plus the column pass in its
 * RK4 stage form (HIP events, `reps` launches each) for each column-pass form
 * (wke_plan_set_column_kernel; the field-parallel form only where it
 * applies, in two workgroup widths: as many lanes as its transforms need,
 * or one product lane per item, each also in half rounds
 * (WKE_COLUMN_FIELDS_HALF); the fused form in the two widths, with its
 * interpolation on the vector units or on the matrix cores) and each
 * candidate number of workgroups that share one column block's quadrature
 * sum (1, 2, 4, ... up to the instance's limit, and the first few counts
 * that make the column pass's tasks a multiple of 256), and keep the
 * fastest; in 3D also the slab pass's workgroup width where two exist.  Results do not depend on the choice beyond rounding.
 * Waits for completion.  us_out (host, may be NULL) receives, per group in
 * order of first appearance of N, the chosen form, the chosen split and its
 * time in microseconds (3 doubles per group). */
wke_status wke_plan_tune(wke_plan_t plan, const double *f, double *Q, int reps, double *us_out);

/* Set the work split by hand: the quadrature sum of every column block is
 * shared by min(n, the instance's limit) workgroups (the limit is one item
 * per item slot, and at least min(N_r N_s, 8) in 2D).  n = 1 keeps each block's sum inside one workgroup; n > 1
 * makes the blocks' workgroups publish partial sums that the last one to
 * finish combines in a fixed order.  Results change only by rounding.
 * Waits for the plan's stream. */
wke_status wke_plan_set_split(wke_plan_t plan, int n);

/* Forms of the column pass (the axis-0 inverse transforms, the products and
 * the weighted sum of Alg. 1).  Item slots: a group of lanes takes one
 * quadrature item and transforms its shifted fields one after another.
 * Field-parallel: every distinct shift vector of a workgroup's items has its
 * own group of lanes and is transformed once, the transformed columns meet
 * in LDS, and the products are taken point by point.  Fused (2D): the
 * field-parallel form, with each workgroup building the slab fields of its
 * own column from the axis-0 spectrum by periodic interpolation along axis
 * 1 (a sum over the row with each slab field's kernel, the inverse DFT of
 * its axis-1 phase row), so that no slab pass runs: one launch per
 * evaluation.  Field-parallel, half rounds: the field-parallel form with
 * each round holding at most half the fields a workgroup can, so that its
 * workgroups are half as large and two share a compute unit (more rounds,
 * less waiting).  Fused on the matrix cores (2D): the fused form with the
 * interpolation sum taken as a real GEMM on 16 x 16 x 4 MFMA tiles (rows
 * j0, columns the slab fields' real and imaginary parts, depth the row
 * index x1 and the real and imaginary parts), its operands read straight
 * into registers.  All forms give the same Q up to rounding. */
enum {
    WKE_COLUMN_SLOTS = 0,
    WKE_COLUMN_FIELDS = 1,
    WKE_COLUMN_FUSED = 2,
    WKE_COLUMN_FIELDS_HALF = 3,
    WKE_COLUMN_FUSED_MFMA = 4
};

/* Choose the column-pass form for every instance of the plan (the default
 * is WKE_COLUMN_FIELDS where it applies, else WKE_COLUMN_SLOTS).  Returns
 * WKE_ERR_UNSUPPORTED, changing nothing, when the field-parallel form is
 * asked for a plan it does not cover (more than 64 product units per item,
 * or one item's distinct shifts not fitting a workgroup, or half of one for
 * WKE_COLUMN_FIELDS_HALF), or the fused form
 * for d = 3 or more than 16 slab fields per instance.  Waits for the plan's
 * stream. */
wke_status wke_plan_set_column_kernel(wke_plan_t plan, int kind);

/* How many shifted fields instance i uses, into counts[3] (host):
 * counts[0] = N_r N_s (1 + N_sig) or N_r N_s (1 + 2 N_sig), the shifts
 * r q-hat, r (q-hat - sigma) / 2 (and r (q-hat + sigma) / 2) of Alg. 1 with
 * c(sigma) = b(-sigma) reused when the sigma rule is antipodal;
 * counts[1] = distinct slab fields (shifts that agree on axes 1..d-1 share
 * the slab pass's transforms); counts[2] = distinct shift vectors (the
 * field-parallel column pass transforms each once per column).  Shifts are
 * taken as equal when they agree to 1e-12 (1 + R). */
wke_status wke_field_counts(wke_plan_t plan, int instance, int *counts);

/* Average device time of each kernel, measured with HIP events on the
 * plan's stream around `reps` back-to-back launches of that kernel on the
 * input f (device, packed grid, only read; Q is written as scratch, and so
 * are the plan's RK4 work arrays).  us_out (host) receives 4 values in
 * microseconds: column forward transform, slab pass (shifted transforms),
 * column pass in its Q form (transforms, products, sums), column pass in
 * its RK4 stage form (the same plus the stage update and the next forward
 * transform).  Caches are warm after the first launch. */
wke_status wke_time_kernels(wke_plan_t plan, const double *f, double *Q, int reps,
                            double *us_out);

/* Algorithmic work of one evaluation of the whole batch, per kernel of
 * wke_time_kernels (column forward, slab pass, column pass): flops_out[3]
 * counts 5 n log2 n per length-n complex transform (the slab pass: one per
 * distinct slab field; the column pass: one per shift, or per distinct
 * shift vector in the field-parallel form) plus the phase multiplies,
 * pointwise products and weighted sums; bytes_out[3] the bytes each kernel
 * must move to or from device memory in this design (its inputs and
 * outputs, the slab fields between the two passes, the phase rows, the
 * partial sums when the quadrature sum is split over workgroups).  Either
 * pointer may be NULL. */
wke_status wke_work_model(wke_plan_t plan, double *flops_out, double *bytes_out);

const char *wke_status_string(wke_status s);
const char *wke_last_error(void);

/* Test hook for the failure paths: after `after` more successful device
 * allocations by this library, the next one fails as if the device were
 * out of memory (the call that needed it returns WKE_ERR_NOMEM and frees
 * what it had allocated); the hook then stays armed at zero until reset.
 * after < 0 switches it off (the default).  Process-wide. */
void wke_test_fail_allocations(int after);

#ifdef __cplusplus
}
#endif

#endif /* WKE_H */

// Shared host/device declarations of the wke library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

#include "wke_types.hpp"

namespace wke {

struct PassBArgs {
    const InstDev* inst;
    const TaskB* tasks;
    const void* G;            // slab fields (T)
    const int* hid;           // slab field of each shift
    const void* ph;           // phase tables (T): each shift's axis-0 factors are applied here
    const RoundDesc* rounds;  // field-parallel form: rounds of each item group
    const FieldRef* flds;         // their distinct fields: (shift whose phases define it, its slab field)
    const int* uofs;          // per item, the LDS offsets of its factors (a, then b and c of each unit)
    void* spec0;              // axis-0 spectrum (T), written in RK mode
    const double* F0;         // current stage state (double2), packed grid
    double* out;              // MODE_EVAL: Q (double2); MODE_RK: unused
    double* y;                // RK base state (double2), written at stage 3
    double* ystage;           // RK stage state (double2)
    double* ksum;             // RK stage-derivative sum (double2)
    const void* uw;           // unit weights (T)
    const UnitPat* upat;      // unit patterns (per instance, U_item entries each)
    const int* upat_off;      // offset of each instance's patterns
    double* part;             // partial sums (double2)
    unsigned int* counters;   // arrival counters
    const void* tw;           // twiddle tables (T)
    int mode, stage;
    double dt;
    int fp_threads;           // > 0: field-parallel column pass with this many threads
    unsigned fp_lds;          // its dynamic LDS bytes
    int fp_fused;             // 2D: build the slab-field columns in the workgroup (no slab pass)
    int fp_nwp;               // fused: chunks of the interpolation sum (matrix-core form: depth splits)
    int fp_mfma;              // fused: the interpolation on the matrix cores
    unsigned fp_off_h;        // fused: LDS byte offset of the slab-field columns
    unsigned fp_off_ph;       // fused: LDS byte offset of the first round's phase rows (0: read from memory)
    const void* kt;           // fused: interpolation kernels (T), [slab field][2N] (each row twice)
    const int* sub;           // fused: slab-field subsets of the item groups ([count, slab field ...] at TaskB::sub)
    int real;                 // Nyquist-zero real form: two real fields per transform, real products
    int one;                  // a single-instance plan with one item group: every task is task1 but for
                              // its column block, which is its place in the list
    TaskB task1;
};

struct PassAArgs {
    const InstDev* inst;
    const TaskA* tasks;
    const void* spec0;        // axis-0 spectrum (T)
    void* G;                  // slab fields (T)
    const void* ph;           // phase tables (T)
    const int* hrep;          // shift whose phase factors (axes 1..d-1) define each slab field
    const void* tw;
    int slab_alt;             // 3D: the alternative workgroup width (Geometry::shifts_per_task_a_alt fields)
};

struct ColFwdArgs {
    const InstDev* inst;
    const TaskB* tasks;       // (inst, cb) pairs
    const double* f;          // packed grid (double2)
    void* spec0;
    const void* tw;
    int spec_trans;           // 2D: store spec0 as [x1][j0] (for the fused column pass)
};

// De-aliased (exact-Galerkin) plans evaluate the operator on the grid of
// P = 2N points and move between the two grids by trigonometric resampling,
// one axis per launch.  One descriptor per instance and launch.
struct ResampleDesc {
    long long in_off, out_off;   // complex offsets of the instance's input and output
    long long n_out;             // output elements of the instance
    long long inner;             // product of the output extents of the axes after the resampled one
    int m_in, m_out;             // extents of the resampled axis before and after (N and P, or P and N)
    int N;                       // coarse size
    int h_off;                   // complex offset of the instance's resampling kernel (N entries)
};
// A classical RK4 stage update (stage 0..3) of the state y with stage
// buffers ys, ks (the exact-Galerkin column kernel's epilogue).
struct RkStage {
    int stage;
    double dt;
    double *y, *ys, *ks;
};

// Root i (descending order) and weight of the n-point Gauss-Legendre rule on
// [-1, 1]: Newton iteration on the three-term Legendre recurrence from
// Tricomi's approximation of the root.
__device__ inline void gl_root(int n, int i, double* xo, double* wo) {
    const double th = M_PI * (4.0 * i + 3.0) / (4.0 * n + 2.0);
    double x = (1.0 - 1.0 / (8.0 * n * n) + 1.0 / (8.0 * n * n * n)) * cos(th);
    double dp = 1.0;
    for (int pass = 0; pass < 101; ++pass) {
        double pm = 1.0, pc = x;   // P_0, P_1
        for (int k = 2; k <= n; ++k) {
            const double pn = ((2.0 * k - 1.0) * x * pc - (k - 1.0) * pm) / k;
            pm = pc;
            pc = pn;
        }
        if (n == 1) { pc = x; pm = 1.0; }
        dp = n * (pm - x * pc) / (1.0 - x * x);
        if (pass == 100) break;      // last pass: the derivative at the final root
        const double dx = pc / dp;
        x -= dx;
        if (fabs(dx) < 1e-17 + 1e-16 * fabs(x)) pass = 99;
    }
    *xo = x;
    *wo = 2.0 / ((1.0 - x * x) * dp * dp);
}

// Exact-weight reference system (wke_exact_system): workspace and sizes.
// Phi(a, b) = sum_k u_k S_a(k) S_b(k) over squared mode norms a <= A, b <= B.
struct ExactArgs {
    int d, N, nr, A, B;
    double L, R;
    double* rk;        // radial nodes on [0, R] (nr)
    double* uk;        // weight times r^(2d-3) (nr)
    double* S;         // sphere means S(pi r_k sqrt(a) / (2L)), [A+1][nr]
    double* phi;       // [A+1][B+1]
    double* F;         // spectrum (double2, N^d)
    double* Qh;        // Q hat (double2, N^d)
    const double* f;   // grid input (double2)
    double* Q;         // grid output (double2)
};
hipError_t launch_exact(const ExactArgs& a, hipStream_t s);
// The allocation-free variant's workspace: a static device array of
// EXACT_SCRATCH_DOUBLES doubles (16 MiB) per GPU.  exact_scratch returns
// its device address on the current device (looked up once per device).
constexpr size_t EXACT_SCRATCH_DOUBLES = (size_t)2 << 20;
constexpr int EXACT_MAX_DEVICES = 64;
hipError_t exact_scratch(double** ptr);

// Launch helpers (defined in wke_kernels.hip).  `prec` is 0 (double) or 1
// (float); N and d select the template instance.  Return hipSuccess or the
// launch error.
hipError_t launch_colfwd(int prec, int d, int N, const ColFwdArgs& a, int ntasks, hipStream_t s);
// Optional start/stop events bound to a dispatch (hipExtLaunchKernel): they
// then time exactly that kernel's execution.
struct LaunchEvents { hipEvent_t start, stop; };
hipError_t launch_passA(int prec, int d, int N, const PassAArgs& a, int ntasks, hipStream_t s,
                        const LaunchEvents* ev = nullptr);
hipError_t launch_passB(int prec, int d, int N, const PassBArgs& a, int ntasks, hipStream_t s,
                        const LaunchEvents* ev = nullptr);
hipError_t launch_tables(const InstDev* inst_dev, const InstDev& inst_host, int inst_index,
                         double* nodes, const UnitPat* upat_dev, double* ph64, float* ph32,
                         double* uw64, float* uw32, hipStream_t s);
hipError_t launch_twiddles(int N, double* tw64, float* tw32, hipStream_t s);
hipError_t launch_ktab(const InstDev* inst_dev, const InstDev& inst_host, int inst_index, const double* ph64,
                       const int* hrep, double* kt64, float* kt32, hipStream_t s);
// Exact-Galerkin RK4 stage on the fine grid (see k_colrk).
struct ColRkArgs {
    const InstDev* inst;      // fine-grid instances
    const TaskB* tasks;       // (inst, cb) pairs, as for the column forward transform
    const double* q;          // fine-grid Q projected along axes 1..d-1 (double2)
    double *y, *ys, *ks;      // fine-grid RK state, stage state, derivative sum (double2)
    void* spec0;              // axis-0 spectrum of the new stage state (T)
    const void* tw64;         // double twiddles (the projection runs in double)
    const void* tw;           // twiddles of T
    int spec_trans, stage;
    double dt;
};
hipError_t launch_colrk(int prec, int d, int N, const ColRkArgs& a, int ntasks, hipStream_t s);

enum { RS_REFINE = 0, RS_COARSEN = 1, RS_PROJECT = 2 };

// Launch shape of one resampling launch: lines per workgroup, workgroups per
// instance (enough for the instance with the most lines), dynamic LDS bytes
// (the largest kernel plus line tile of the batch).
struct ResampleLaunch { int lt; int blocks; unsigned lds; };
// kind RS_REFINE (N -> P), RS_COARSEN (P -> N) or RS_PROJECT (P -> P) along
// the axis the descriptors name.
hipError_t launch_resample(int kind, const ResampleDesc* rd, int batch, const ResampleLaunch& g, const double* h,
                           const double* in, double* out, hipStream_t s);
// Even fine-grid samples onto the coarse grid; rd gives out_off and N per
// instance, fine_off (device) the fine offsets; n_max the largest N.
hipError_t launch_decimate(const ResampleDesc* rd, const long long* fine_off, int batch, int d, int n_max,
                           const double* in, double* out, hipStream_t s);
hipError_t launch_moments(const InstDev* inst, int batch, const double* f, double* out, hipStream_t s);
// In place: the grid function at data (double2, [N]^d) becomes its Fourier
// coefficients in FFT index order (d launches, one per axis).  N must be one
// of 8, 16, 32, 48, 64, 96, 128 (hipErrorInvalidValue otherwise).
hipError_t launch_spectrum(int d, int N, double* data, hipStream_t s);

}  // namespace wke

// Plain C++ types shared by the kernels and the host-side plan layout (no
// HIP dependency, so the layout code also builds as ordinary host C++).
#pragma once

namespace wke {

// Per-instance descriptor, resident in device memory.
struct InstDev {
    int d, N, Nr, Ns, Nsig, rule;
    int antipodal;      // 1 if the sigma rule is closed under sigma -> -sigma
    int S_item;         // shifted fields per (p1, p2) item: a, then b's (and c's)
    int U_item;         // product units per item
    int n_items;        // N_r * N_s
    int n_shift;        // n_items * S_item
    int n_slab;         // distinct slab fields: shifts with equal components on axes 1..d-1 share one
    int n_unit;         // n_items * U_item
    int n_ig;           // item groups of the column pass (partial sums)
    int items_per_ig;
    int n_cb;           // column blocks of the column pass
    int counter_off;    // first arrival counter of this instance
    int nyq_zero;       // 1: the Nyquist-zero real form (every mode with a component -N/2 dropped from the
                        // operator's input, Re f only); its phase tables carry one more row, the zero shift
    double L, R, h;
    double fwd_scale;   // 1 / N^d
    double q_scale;     // 2^(1-d)
    long long n_pts;    // N^d
    long long off_state;   // complex offset in packed grid arrays
    long long off_spec0;   // complex offset in the axis-0 spectrum workspace
    long long off_G;       // complex offset in the slab-field workspace (n_slab fields)
    long long off_hrep;    // offset of this instance's slab-field representatives (shift index per slab field)
    long long off_hid;     // offset of this instance's per-shift tables (slab field; round-local field)
    long long off_rounds;  // offset of this instance's rounds (field-parallel column pass)
    long long off_kt;      // offset of this instance's axis-1 interpolation kernels (2D, n_slab x 2N: each row twice)
    long long off_nodes;   // double offset of r, wr, qh, ws, sg, wsig
    long long off_ph;      // complex offset of this instance's phase tables
    long long off_unit;    // offset of this instance's units
    long long off_part;    // complex offset in the partial-sum workspace
    long long off_tw;      // complex offset of the twiddle table of N
};

struct UnitPat {        // one product unit of an item
    int b;              // shift index (within the item) of the factor b
    int c;              // shift index of the factor c
    int p3, p3b;        // sigma node(s) whose weights the unit carries (-1: none)
};

// A column-pass workgroup stages the slab-field index of each shift of its
// items in LDS: at most HID_CAP of them (the host splits the items to fit).
constexpr int HID_CAP = 1024;

struct TaskA { int inst, j0, s_begin, s_end; };   // slab-pass task: slab j0, slab fields [s_begin, s_end)
// Column-pass task: column block cb, item group ig.  The field-parallel form
// also reads its rounds [r0, r1) and their field list (nfl entries from f0);
// the fused form the slab fields its items use: sub is the offset of
// [count, slab field ...] in the plan's subset table.
struct TaskB { int inst, cb, ig, r0, r1, f0, nfl, sub; };
// A distinct field of a round: the shift whose phases define it and its
// slab field.
struct FieldRef { int x, y; };
// One round of the field-parallel column pass: items [ia, ib) whose shifts
// use the nf distinct fields listed from foff.
struct RoundDesc { int ia, ib, foff, nf; };

// Evaluation modes of the column pass epilogue.
enum { MODE_EVAL = 0, MODE_RK = 1 };

// Field-parallel column pass: static limits of one workgroup (weights of a
// round's (item, unit) pairs, product units of an item), the columns a
// workgroup covers in dimension d, the most distinct fields it can hold at
// once for (prec, d, N), the threads that carry ng fields with (up to) kp
// product lanes per grid point (0 if even one lane per point does not fit),
// and the dynamic LDS bytes of a launch with nt threads and ng fields.
constexpr int FP_MAX_GROUPS = 256, FP_MAX_UNITS = 64;
int fp_columns(int d);
int fp_group_cap(int prec, int d, int N, bool fused = false, bool real = false);
int fp_threads(int prec, int d, int N, int ng, int kp, bool fused = false, bool real = false);
unsigned fp_lds_bytes(int prec, int d, int N, int nt, int ng);
// Fused 2D form: at most FUSED_MAX_SLAB slab fields; the chunks of the
// interpolation sum for nt threads (0: the form does not fit); the dynamic
// LDS bytes (and the offset of the slab-field columns) with ns slab fields.
constexpr int FUSED_MAX_SLAB = 16;
int fused_chunks(int prec, int N, int nt);
// nparts: the partial sums of the interpolation ([part][slab field][j0]):
// fused_chunks for the vector form, the depth splits for the matrix-core form
unsigned fused_lds_bytes(int prec, int N, int nt, int ng, int ns, int nparts, unsigned* off_h);

// Geometry of the template instances (threads per block, groups, LDS bytes).
// groups_a: rows per 2D slab-pass task (JB; 1 in 3D); shifts_per_task_a:
// shifted fields per slab-pass task; groups_b x slots_b: columns x item slots
// of a column-pass workgroup; groups_f: columns per column-forward workgroup.
// shifts_per_task_a_alt: the alternative 3D slab-pass workgroup width, in
// fields transformed at once (0: none).
struct Geometry { int tpt, groups_a, groups_b, slots_b, groups_f, shifts_per_task_a, shifts_per_task_a_alt; };
bool geometry_of(int prec, int d, int N, Geometry* g);   // prec: 0 double, 1 float

}  // namespace wke

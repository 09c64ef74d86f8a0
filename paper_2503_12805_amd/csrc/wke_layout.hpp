// Host-side layout of a plan: per-instance descriptors and table offsets,
// shared slab fields and distinct shift vectors, work splits, the
// field-parallel rounds and the task lists of every launch.  Plain C++ (no
// HIP): the library calls it between its device steps, and a CPU test
// builds it on its own, with address and undefined-behaviour sanitizers,
// to check every offset and range it produces.
#pragma once

#include <map>
#include <string>
#include <vector>

#include "wke.h"
#include "wke_types.hpp"

namespace wke {

struct Group {              // instances sharing one grid size N
    int N = 0;
    int colkind = 0;        // column pass: 0 item slots, 1 field-parallel, 2 fused (2D, no slab pass)
    int fp_wide = 0;        // field-parallel: one product lane per item (up to 16 per point), else fewest lanes
    int fp_half = 0;        // field-parallel: rounds of at most half the fields a workgroup can hold, so that
                            // two workgroups share a compute unit
    int fp_threads = 0;     // field-parallel launch: threads and dynamic LDS bytes
    unsigned fp_lds = 0;
    unsigned fp_off_h = 0;  // fused: LDS offset of the slab-field columns
    unsigned fp_off_ph = 0; // fused: LDS offset of the first round's phase rows (0: none)
    int slab_alt = 0;       // 3D slab pass in its alternative workgroup width (the starting choice for
                            // some single-instance groups, or the autotuner's)
    int fp_nwp = 0;         // fused: chunks of the interpolation sum (matrix-core form: depth splits)
    int fp_mfma = 0;        // fused: the interpolation on the matrix cores
    std::vector<TaskA> hA;  // slab-pass tasks
    std::vector<TaskB> hB;  // column-pass tasks of the current split
    std::vector<TaskB> hF;  // column forward-transform tasks
    size_t maxB = 0;        // most column-pass tasks any split can need (device list capacity)
    size_t maxA = 0;        // most slab-pass tasks either workgroup width can need (device list capacity)
    TaskA* dA = nullptr;    // device copies, owned by the plan
    TaskB* dB = nullptr;
    TaskB* dF = nullptr;
};

struct PlanLayout {
    int batch = 0, prec = 0, d = 0;
    int nyq = 0;                       // Nyquist-zero real form
    std::vector<wke_desc> desc;
    std::vector<InstDev> inst;
    std::vector<std::vector<UnitPat>> pats;
    std::vector<int> pat_off;          // offset of each instance's unit patterns
    std::vector<int> max_ig;           // largest useful split of each instance's quadrature sum
    std::vector<int> min_ig;           // smallest split whose items' slab-field indices fit a workgroup
    std::vector<std::vector<int>> hrep, hid;   // slab-field representatives and slab field of each shift
    std::vector<std::vector<int>> fid, frep;   // distinct shift vectors: id of each shift, representatives
    // field-parallel rounds for the current split, per instance
    std::vector<std::vector<RoundDesc>> rounds;
    std::vector<std::vector<FieldRef>> flds;
    std::vector<std::vector<int>> lidx;
    // per item, in the S_item = 1 + 2 U_item entries of its shifts: the
    // column pass's LDS offsets (from a point's own slot) of its factor a and
    // of b and c of each unit, in unit order (what the kernel reads; lidx
    // keeps the round-local field of each shift)
    std::vector<std::vector<int>> uofs;
    std::vector<std::vector<int>> ig_r0, ig_r1, ig_f0, ig_nfl;
    // fused form: per item group, the slab fields its rounds use (the
    // rounds' fields then name them by their place in this list); all
    // groups' lists back to back as [count, slab field ...], and each item
    // group's offset into that table
    std::vector<int> sub;
    std::vector<std::vector<int>> ig_sub;
    std::vector<long long> sub_off;    // each instance's region of the table
    std::vector<int> rounds_fused;     // 1 where an instance's rounds name subset places
    std::vector<int> fp_ns;            // most slab fields one workgroup interpolates (fused form)
    long long n_sub = 0;               // size of the subset table
    std::vector<int> fp_ng;            // most fields of one round
    std::vector<int> fp_ni;            // most items of one round
    std::vector<Group> groups;
    std::map<int, long long> tw_off;   // N -> complex offset in the twiddle tables
    size_t total_elems = 0;
    // sizes of the plan's tables (elements of their type)
    long long n_spec0 = 0, n_G = 0, n_part = 0, n_nodes = 0, n_ph = 0, n_unit = 0, n_tw = 0;
    long long n_hrep = 0, n_hid = 0, n_rounds = 0, n_kt = 0;
    int n_counters = 0;
};

// Descriptor checks (before anything is allocated); WKE_OK or an error
// status with a message in *err.
wke_status validate_descs(const wke_desc* insts, int batch, int precision, std::string* err);
bool supported_N(int d, int N);
int rule_points(int rule);
// Index of the antipode of sigma node p3 in the rule's ordering, or -1.
int antipode(int d, int rule, int n, int p3);

// Step 1: instance descriptors, unit patterns, work-split bounds and every
// offset that does not depend on the quadrature nodes.
void layout_instances(PlanLayout* L, const wke_desc* insts, int batch, int precision, int nyq);
// Step 2, with the quadrature nodes (layout r, wr, q-hat, w_s, sigma,
// w_sigma per instance at inst[i].off_nodes): shared slab fields, distinct
// shift vectors and the offsets and sizes of the tables they index.
void layout_fields(PlanLayout* L, const double* nodes);
// Step 3: per N group, the slab-pass and column-forward tasks, the column
// form and width to start with, and the column-pass task capacity.
void layout_tasks(PlanLayout* L);
// Slab-pass tasks of group G in the default (alt = 0) or the alternative
// (alt = 1) 3D workgroup width, or (alt < 0) the plan's starting choice;
// whether an alternative width exists for G.
void layout_slab_tasks(PlanLayout* L, Group& G, int alt);
bool slab_alt_available(const PlanLayout* L, const Group& G);
// Column-pass tasks and field-parallel rounds of group G under the current
// splits (set_split) and form (G.colkind, G.fp_wide, G.fp_half).
void layout_split(PlanLayout* L, Group& G);

void set_split(PlanLayout* L, int i, int n);
int fp_field_cap(const PlanLayout* L, int N, int half = 0, bool fused = false);
bool fp_feasible(const PlanLayout* L, const Group& G, int half = 0, bool fused = false);
void update_fp(PlanLayout* L, Group& G);
bool fused_width_ok(PlanLayout* L, Group& G, int wide, int mfma = 0);
bool fused_feasible(PlanLayout* L, Group& G, int mfma = 0);

// Whether the column-pass launch shape of group G (after layout_split)
// fits its kernel: lanes for the field blocks within the workgroup limit,
// the dynamic LDS within its limit, and, in the fused form, a chunking of
// the interpolation sum.  A form and split that do not fit are refused.
bool launch_fits(const Group& G);

// Every offset and range of the layout against the table sizes, every task
// and round against the lists it indexes, and every launch shape against
// its limits.  Returns "" if all hold, else the first violation found.
std::string check_layout(const PlanLayout& L);

}  // namespace wke

// Host side of the wke library: plan construction, workspace, dispatch, and
// the C interface declared in include/wke.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdarg>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "wke.h"
#include "wke_internal.hpp"

using namespace wke;

namespace {

thread_local std::string g_last_error;

wke_status fail(wke_status s, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
wke_status fail(wke_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return s;
}

#define HIP_TRY(call)                                                                          \
    do {                                                                                       \
        hipError_t e_ = (call);                                                                \
        if (e_ != hipSuccess)                                                                  \
            return fail(WKE_ERR_HIP, "%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), __FILE__, \
                        __LINE__);                                                             \
    } while (0)

struct Group {          // instances sharing one grid size N
    int N = 0;
    int colkind = 0;        // column pass: 0 item slots, 1 field-parallel, 2 fused (2D, no slab pass)
    int fp_wide = 0;        // field-parallel: one product lane per item (up to 16 per point), else fewest lanes
    int fp_half = 0;        // field-parallel: rounds of at most half the fields a workgroup can hold, so that
                            // two workgroups share a compute unit
    int fp_threads = 0;     // field-parallel launch: threads and dynamic LDS bytes
    unsigned fp_lds = 0;
    unsigned fp_off_h = 0;  // fused: LDS offset of the slab-field columns
    unsigned fp_off_ph = 0; // fused: LDS offset of the first round's phase rows (0: none)
    int slab_alt = 0;       // 3D slab pass in its wider workgroup (single-instance groups)
    int fp_nwp = 0;         // fused: chunks of the interpolation sum
    std::vector<TaskA> hA;
    std::vector<TaskB> hB, hF;
    TaskA* dA = nullptr;
    TaskB* dB = nullptr;
    TaskB* dF = nullptr;
};

}  // namespace

struct wke_plan_s {
    int batch = 0, prec = 0, d = 0;
    int nyq = 0;                       // Nyquist-zero real form (wke_plan_create_real)
    hipStream_t stream = nullptr;
    int device = 0;
    std::vector<wke_desc> desc;
    std::vector<InstDev> inst;
    std::vector<std::vector<UnitPat>> pats;
    std::vector<int> max_ig;           // largest useful split of each instance's quadrature sum
    std::vector<int> min_ig;           // smallest split whose items' slab-field indices fit a workgroup
    std::vector<std::vector<int>> hrep, hid;   // slab-field representatives and slab field of each shift
    std::vector<std::vector<int>> fid, frep;   // distinct shift vectors: id of each shift, representatives
    // field-parallel rounds for the current split, per instance
    std::vector<std::vector<RoundDesc>> rounds;
    std::vector<std::vector<int2>> flds;
    std::vector<std::vector<int>> lidx;
    std::vector<std::vector<int>> ig_r0, ig_r1, ig_f0, ig_nfl;
    std::vector<int> fp_ng;            // most fields of one round
    std::vector<int> fp_ni;            // most items of one round
    std::vector<Group> groups;
    std::map<int, long long> tw_off;   // N -> complex offset in the twiddle tables
    size_t total_elems = 0;
    long long n_spec0 = 0, n_G = 0, n_part = 0, n_nodes = 0, n_ph = 0, n_unit = 0, n_tw = 0;
    int n_counters = 0;
    // device memory
    InstDev* d_inst = nullptr;
    double* d_nodes = nullptr;
    UnitPat* d_upat = nullptr;
    int* d_upat_off = nullptr;
    double* d_ph64 = nullptr;
    float* d_ph32 = nullptr;
    double* d_uw64 = nullptr;
    float* d_uw32 = nullptr;
    double* d_tw64 = nullptr;
    float* d_tw32 = nullptr;
    void* d_spec0 = nullptr;
    void* d_G = nullptr;
    double* d_part = nullptr;
    unsigned int* d_counters = nullptr;
    double* d_ystage = nullptr;
    double* d_ksum = nullptr;
    double* d_mom = nullptr;
    int* d_hrep = nullptr;
    int* d_hid = nullptr;
    RoundDesc* d_rounds = nullptr;
    int2* d_flds = nullptr;
    int* d_lidx = nullptr;
    double* d_kt64 = nullptr;          // 2D axis-1 interpolation kernels of the slab fields
    float* d_kt32 = nullptr;
    std::vector<void*> allocs;
    // one captured RK4 step (8 kernel launches) replayed by wke_step
    bool use_graphs = false;
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t step_exec = nullptr;
    const double* graph_f = nullptr;
    double graph_dt = 0.0;
    // exact-Galerkin (de-aliased) plans: the operator runs on `fine`, a plan
    // over the grids of 2N points; this plan keeps the coarse layout, the
    // RK4 stage buffers and the resampling between the two
    wke_plan_s* fine = nullptr;
    double* d_fP = nullptr;            // fine-grid state (fine packing)
    double* d_QP = nullptr;            // fine-grid Q
    double* d_ysP = nullptr;           // fine-grid RK4 stage state and derivative sum
    double* d_ksP = nullptr;
    long long* d_fine_off = nullptr;   // fine offset of each instance
    double* d_t1 = nullptr;            // resampling intermediates (fine packing)
    double* d_t2 = nullptr;
    double* d_hres = nullptr;          // resampling kernels, N per instance
    ResampleDesc* d_rs = nullptr;      // [refining axes d, coarsening axes d, projecting axes d-1][batch]
    std::vector<ResampleLaunch> rs_launch;   // launch shape of each of those launches
};

namespace {

wke_status apply_split(wke_plan_s* p, Group& G);

bool supported_N(int d, int N) {
    Geometry g;
    return geometry_of(0, d, N, &g);
}

int rule_points(int rule) {
    switch (rule) {
        case WKE_OCTAHEDRON: return 6;
        case WKE_CUBE: return 8;
        case WKE_ICOSAHEDRON: return 12;
    }
    return 0;
}

// Index of the antipode of sigma node p3 in the rule's ordering, or -1 when
// the rule is not closed under sigma -> -sigma.
int antipode(int d, int rule, int n, int p3) {
    if (d == 2) {
        if (n % 2) return -1;             // (2i+1) pi / n + pi is a node only for even n
        return (p3 + n / 2) % n;
    }
    switch (rule) {
        case WKE_OCTAHEDRON: return p3 ^ 1;    // +e_a, -e_a adjacent
        case WKE_CUBE: return 7 - p3;          // all three sign bits flipped
        case WKE_ICOSAHEDRON: return p3 ^ 3;   // both signs flipped, same cyclic shift
    }
    return -1;
}

// Every device allocation of the library goes through here.  Test hook
// (wke_test_fail_allocations): with a budget b >= 0, b more allocations
// succeed and the next one fails as if the device were out of memory,
// without calling the runtime.
std::atomic<long> g_alloc_budget{-1};

hipError_t alloc_device(void** q, size_t bytes) {
    *q = nullptr;
    long b = g_alloc_budget.load();
    while (b >= 0) {
        if (b == 0) return hipErrorOutOfMemory;
        if (g_alloc_budget.compare_exchange_weak(b, b - 1)) break;
    }
    const hipError_t e = hipMalloc(q, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();    // clear the runtime's sticky error of the failed call
        *q = nullptr;
    }
    return e;
}

template <class X> wke_status dev_alloc(wke_plan_s* p, X** ptr, size_t count) {
    *ptr = nullptr;
    if (count == 0) count = 1;
    void* q = nullptr;
    hipError_t e = alloc_device(&q, count * sizeof(X));
    if (e != hipSuccess)
        return fail(WKE_ERR_NOMEM, "device allocation of %zu bytes failed: %s", count * sizeof(X),
                    hipGetErrorString(e));
    p->allocs.push_back(q);
    *ptr = static_cast<X*>(q);
    return WKE_OK;
}

#define WKE_TRY(x)                     \
    do {                               \
        wke_status s_ = (x);           \
        if (s_ != WKE_OK) return s_;   \
    } while (0)

wke_status validate(const wke_desc* insts, int batch, int precision) {
    if (!insts || batch < 1) return fail(WKE_ERR_INVALID, "need at least one instance");
    if (precision != WKE_F64 && precision != WKE_F32) return fail(WKE_ERR_INVALID, "precision must be WKE_F64 or WKE_F32");
    const int d0 = insts[0].d;
    for (int i = 0; i < batch; ++i) {
        const wke_desc& q = insts[i];
        if (q.d != 2 && q.d != 3) return fail(WKE_ERR_INVALID, "instance %d: d must be 2 or 3", i);
        if (q.d != d0) return fail(WKE_ERR_INVALID, "instance %d: all instances of a plan must share d", i);
        if (q.N < 2 || (q.N & 1)) return fail(WKE_ERR_INVALID, "instance %d: N must be even and >= 2", i);
        if (!supported_N(q.d, q.N)) return fail(WKE_ERR_UNSUPPORTED, "instance %d: N = %d is not built for d = %d", i, q.N, q.d);
        if (!(q.L > 0.0) || !std::isfinite(q.L)) return fail(WKE_ERR_INVALID, "instance %d: L must be positive", i);
        if (!std::isfinite(q.R)) return fail(WKE_ERR_INVALID, "instance %d: R must be finite", i);
        if (q.N_r < 1 || q.N_s < 1 || q.N_sig < 1) return fail(WKE_ERR_INVALID, "instance %d: quadrature counts must be >= 1", i);
        if (q.N_r > 4096) return fail(WKE_ERR_INVALID, "instance %d: N_r too large", i);
        if (q.d == 2) {
            if (q.sphere_rule != WKE_MIDPOINT) return fail(WKE_ERR_INVALID, "instance %d: 2D uses WKE_MIDPOINT", i);
            if (q.N_s > 4096 || q.N_sig > 4096) return fail(WKE_ERR_INVALID, "instance %d: angle counts too large", i);
        } else {
            const int np = rule_points(q.sphere_rule);
            if (!np) return fail(WKE_ERR_INVALID, "instance %d: 3D needs a spherical design rule", i);
            if (q.N_s != np || q.N_sig != np)
                return fail(WKE_ERR_INVALID, "instance %d: N_s and N_sig must equal the design's %d points", i, np);
        }
        const double R = q.R > 0 ? q.R : 4.0 * q.L / (3.0 + std::sqrt(2.0));
        if (R > 2.0 * q.L) return fail(WKE_ERR_INVALID, "instance %d: R must not exceed 2L", i);
    }
    return WKE_OK;
}

// Shift vector number ls of an instance, from its quadrature nodes (layout
// r, wr, q-hat, w_s, sigma, w_sigma): s_a = r q-hat, s_b = r (q-hat - sigma) / 2,
// s_c = r (q-hat + sigma) / 2, the same expressions the phase tables use.
void shift_vector(const InstDev& I, const double* nd, int ls, double* s) {
    const int d = I.d;
    if (ls >= I.n_shift) {                 // the real form's extra row: the zero shift
        for (int a = 0; a < d; ++a) s[a] = 0.0;
        return;
    }
    const double* r = nd;
    const double* qh = nd + 2 * I.Nr;
    const double* sg = qh + I.Ns * (d + 1);
    const int it = ls / I.S_item, k = ls % I.S_item;
    const int p1 = it / I.Ns, p2 = it % I.Ns;
    for (int a = 0; a < d; ++a) {
        const double q = qh[p2 * d + a];
        if (k == 0) s[a] = r[p1] * q;
        else if (k <= I.Nsig) s[a] = 0.5 * r[p1] * (q - sg[(k - 1) * d + a]);
        else s[a] = 0.5 * r[p1] * (q + sg[(k - 1 - I.Nsig) * d + a]);
    }
}

// Shifts whose components on axes 1..d-1 agree (to a few units of rounding)
// have the same slab field: the slab pass applies only those axes' phase
// factors.  hrep[h] is the first shift of slab field h, hid[ls] the slab
// field of shift ls.  The symmetric sphere rules make many shifts agree: for
// the 4-point midpoint rule the 2D shifts of one radius take 3 distinct
// axis-1 components, the cube design's 3D shifts 9 distinct pairs.
// With a0 = 0 instead of 1 the same grouping finds the distinct shift
// vectors themselves (the fields of the column pass).
void group_shifts(const InstDev& I, const double* nd, int a0, std::vector<int>* hrep, std::vector<int>* hid) {
    const double tol = 1e-12 * (1.0 + I.R);
    std::map<std::vector<long long>, int> seen;
    hrep->clear();
    const int n = I.n_shift + I.nyq_zero;     // with the real form's zero shift
    hid->assign(n, 0);
    double sv[3];
    for (int ls = 0; ls < n; ++ls) {
        shift_vector(I, nd, ls, sv);
        std::vector<long long> key;
        for (int a = a0; a < I.d; ++a) key.push_back(std::llround(sv[a] / tol));
        auto it = seen.find(key);
        if (it == seen.end()) {
            it = seen.emplace(key, (int)hrep->size()).first;
            hrep->push_back(ls);
        }
        (*hid)[ls] = it->second;
    }
}

// Columns per workgroup of the item-slot column pass.
int g_slots_columns(int prec, int d, int N) {
    Geometry g;
    geometry_of(prec, d, N, &g);
    return g.groups_b;
}

// The field-parallel column pass needs few enough product units per item and
// room for one item's fields in a workgroup.
// Distinct fields a field-parallel workgroup holds at once: one per lane
// block, two in the real form (real and imaginary part of one column).
int fp_field_cap(const wke_plan_s* p, int N, int half = 0) {
    const int g = fp_group_cap(p->prec, p->d, N);
    return (half ? g / 2 : g) * (p->nyq ? 2 : 1);
}

bool fp_feasible(const wke_plan_s* p, const Group& G, int half = 0) {
    const int cap = fp_field_cap(p, G.N, half);
    for (const InstDev& I : p->inst) {
        if (I.N != G.N) continue;
        // every round of the real form also holds the zero shift
        if (I.U_item > FP_MAX_UNITS || I.S_item + I.nyq_zero > cap || I.n_items * I.U_item <= 0) return false;
    }
    return cap > 0;
}

// Launch shape of the field-parallel column pass for the group's current
// work split: enough lane groups for one item group's fields (in rounds of
// whole items when they do not fit).
void update_fp(wke_plan_s* p, Group& G) {
    G.fp_threads = 0;
    G.fp_lds = 0;
    G.fp_off_h = 0;
    G.fp_off_ph = 0;
    G.fp_nwp = 0;
    if (G.colkind == 0) return;
    int ng = 0, ni = 0;
    for (int i = 0; i < p->batch; ++i)
        if (p->inst[i].N == G.N) {
            ng = std::max(ng, p->fp_ng[i]);
            ni = std::max(ni, p->fp_ni[i]);
        }
    // wide: enough product lanes per point for one item each (up to 16),
    // for few, latency-bound workgroups; narrow: as few lanes as the
    // transforms need, for batches with many workgroups per compute unit
    if (p->nyq) ng = (ng + 1) / 2;         // lane blocks: two fields each in the real form
    G.fp_threads = fp_threads(p->prec, p->d, G.N, ng, G.fp_wide ? std::min(16, std::max(1, ni)) : 1);
    G.fp_lds = fp_lds_bytes(p->prec, p->d, G.N, G.fp_threads, ng);
    if (G.colkind == 2) {
        int ns = 0;
        for (int i = 0; i < p->batch; ++i)
            if (p->inst[i].N == G.N) ns = std::max(ns, p->inst[i].n_slab);
        G.fp_nwp = fused_chunks(p->prec, G.N, G.fp_threads);
        G.fp_lds = fused_lds_bytes(p->prec, G.N, G.fp_threads, ng, ns, &G.fp_off_h);
        // the first round's phase rows, one (real form: two) per lane block
        const unsigned stage = (unsigned)(ng * (p->nyq ? 2 : 1) * G.N * (p->prec == WKE_F64 ? 16 : 8));
        if (G.fp_lds + stage <= 140 * 1024) {
            G.fp_off_ph = G.fp_lds;
            G.fp_lds += stage;
        }
    }
}

// The fused 2D form also needs few slab fields, a chunking of the
// interpolation sum and its LDS within bounds, at the given width.
bool fused_width_ok(wke_plan_s* p, Group& G, int wide) {
    if (p->d != 2 || !fp_feasible(p, G)) return false;
    for (const InstDev& I : p->inst)
        if (I.N == G.N && I.n_slab > FUSED_MAX_SLAB) return false;
    const int kind = G.colkind, w0 = G.fp_wide;
    G.colkind = 2;
    G.fp_wide = wide;
    update_fp(p, G);
    const bool ok = G.fp_threads > 0 && G.fp_nwp > 0 && G.fp_lds <= 140 * 1024;
    G.colkind = kind;
    G.fp_wide = w0;
    update_fp(p, G);
    return ok;
}

bool fused_feasible(wke_plan_s* p, Group& G) { return fused_width_ok(p, G, 1) || fused_width_ok(p, G, 0); }

wke_status build_plan(wke_plan_s* p, const wke_desc* insts, int batch, int precision) {
    p->batch = batch;
    p->prec = precision;
    p->d = insts[0].d;
    p->desc.assign(insts, insts + batch);
    HIP_TRY(hipGetDevice(&p->device));
    const size_t tsz = precision == WKE_F64 ? 16 : 8;   // bytes per complex value of the compute type
    (void)tsz;

    // distinct N values, in order of first appearance
    std::vector<int> Ns;
    for (int i = 0; i < batch; ++i)
        if (std::find(Ns.begin(), Ns.end(), insts[i].N) == Ns.end()) Ns.push_back(insts[i].N);
    for (int N : Ns) {
        p->tw_off[N] = p->n_tw;
        p->n_tw += N;
    }

    int total_pass_b_cb = 0;
    for (int i = 0; i < batch; ++i) {
        Geometry g;
        geometry_of(precision, insts[i].d, insts[i].N, &g);
        const long long C = insts[i].d == 2 ? insts[i].N : (long long)insts[i].N * insts[i].N;
        total_pass_b_cb += (int)((C + g.groups_b - 1) / g.groups_b);
    }

    p->inst.resize(batch);
    p->pats.resize(batch);
    p->max_ig.assign(batch, 1);
    p->min_ig.assign(batch, 1);
    long long off_state = 0;
    int counter_off = 0;
    for (int i = 0; i < batch; ++i) {
        const wke_desc& q = insts[i];
        InstDev& I = p->inst[i];
        std::memset(&I, 0, sizeof I);
        Geometry g;
        geometry_of(precision, q.d, q.N, &g);
        I.d = q.d;
        I.N = q.N;
        I.Nr = q.N_r;
        I.Ns = q.N_s;
        I.Nsig = q.N_sig;
        I.rule = q.sphere_rule;
        I.L = q.L;
        I.R = q.R > 0 ? q.R : 4.0 * q.L / (3.0 + std::sqrt(2.0));
        I.h = 2.0 * q.L / q.N;
        long long np = 1;
        for (int a = 0; a < q.d; ++a) np *= q.N;
        I.n_pts = np;
        I.fwd_scale = 1.0 / (double)np;
        I.q_scale = std::ldexp(1.0, 1 - q.d);
        // antipodal pairing of sigma nodes
        bool anti = true;
        for (int p3 = 0; p3 < q.N_sig; ++p3)
            if (antipode(q.d, q.sphere_rule, q.N_sig, p3) < 0) anti = false;
        I.antipodal = anti ? 1 : 0;
        std::vector<UnitPat>& pat = p->pats[i];
        if (anti) {
            // c(sigma) = b(-sigma): one b field per sigma, one unit per pair
            I.S_item = 1 + q.N_sig;
            for (int p3 = 0; p3 < q.N_sig; ++p3) {
                const int pa = antipode(q.d, q.sphere_rule, q.N_sig, p3);
                if (p3 < pa) pat.push_back(UnitPat{1 + p3, 1 + pa, p3, pa});
            }
        } else {
            I.S_item = 1 + 2 * q.N_sig;
            for (int p3 = 0; p3 < q.N_sig; ++p3) pat.push_back(UnitPat{1 + p3, 1 + q.N_sig + p3, p3, -1});
        }
        I.U_item = (int)pat.size();
        I.n_items = q.N_r * q.N_s;
        I.n_shift = I.n_items * I.S_item;
        I.n_unit = I.n_items * I.U_item;
        const long long C = q.d == 2 ? q.N : (long long)q.N * q.N;
        I.n_cb = (int)((C + g.groups_b - 1) / g.groups_b);
        // split the quadrature sum over enough workgroups to fill the chip,
        // but give every item slot of a workgroup at least one item; the
        // field-parallel 2D form may split further (up to 8 groups)
        const int slot_ig = std::max(1, (I.n_items + g.slots_b - 1) / g.slots_b);
        // a workgroup stages its items' slab-field indices in LDS (HID_CAP)
        // (the real form adds the zero shift to every round's fields)
        const int s_cap = HID_CAP / (I.S_item + p->nyq);
        const int min_ig = (I.n_items + s_cap - 1) / s_cap;
        const int max_ig = std::max(min_ig, q.d == 2 ? std::max(slot_ig, std::min(I.n_items, 8)) : slot_ig);
        p->max_ig[i] = max_ig;
        p->min_ig[i] = min_ig;
        const int want = std::max(1, (256 + total_pass_b_cb - 1) / total_pass_b_cb);
        I.n_ig = std::max(min_ig, std::min(slot_ig, want));
        I.items_per_ig = (I.n_items + I.n_ig - 1) / I.n_ig;
        I.n_ig = (I.n_items + I.items_per_ig - 1) / I.items_per_ig;
        I.counter_off = counter_off;
        counter_off += (int)C;          // room for one arrival counter per column
        I.off_state = off_state;
        I.off_spec0 = off_state;
        off_state += np;
        I.off_nodes = p->n_nodes;
        p->n_nodes += 2LL * q.N_r + (long long)(q.d + 1) * (q.N_s + q.N_sig);
        I.nyq_zero = p->nyq;
        I.off_ph = p->n_ph;
        p->n_ph += (long long)(I.n_shift + p->nyq) * q.d * q.N;
        I.off_unit = p->n_unit;
        p->n_unit += I.n_unit;
        I.off_part = p->n_part;
        if (max_ig > 1) p->n_part += (long long)max_ig * np;   // room for any split
        I.off_tw = p->tw_off[q.N];
    }
    p->total_elems = (size_t)off_state;
    p->n_spec0 = off_state;
    p->n_counters = counter_off;

    for (int N : Ns) {
        Group G;
        G.N = N;
        p->groups.push_back(std::move(G));
    }

    // device allocations
    WKE_TRY(dev_alloc(p, &p->d_inst, batch));
    WKE_TRY(dev_alloc(p, &p->d_nodes, p->n_nodes));
    size_t npat = 0;
    std::vector<int> pat_off(batch);
    for (int i = 0; i < batch; ++i) {
        pat_off[i] = (int)npat;
        npat += p->pats[i].size();
    }
    WKE_TRY(dev_alloc(p, &p->d_upat, npat));
    WKE_TRY(dev_alloc(p, &p->d_upat_off, batch));
    WKE_TRY(dev_alloc(p, &p->d_ph64, 2 * p->n_ph));
    WKE_TRY(dev_alloc(p, &p->d_uw64, p->n_unit));
    if (precision == WKE_F32) {
        WKE_TRY(dev_alloc(p, &p->d_ph32, 2 * p->n_ph));
        WKE_TRY(dev_alloc(p, &p->d_uw32, p->n_unit));
    }
    WKE_TRY(dev_alloc(p, &p->d_tw64, 2 * p->n_tw));
    WKE_TRY(dev_alloc(p, &p->d_tw32, 2 * p->n_tw));
    if (precision == WKE_F64) {
        double* a;
        WKE_TRY(dev_alloc(p, &a, 2 * p->n_spec0));
        p->d_spec0 = a;
    } else {
        float* a;
        WKE_TRY(dev_alloc(p, &a, 2 * p->n_spec0));
        p->d_spec0 = a;
    }
    WKE_TRY(dev_alloc(p, &p->d_part, 2 * std::max<long long>(1, p->n_part)));
    WKE_TRY(dev_alloc(p, &p->d_counters, std::max(1, p->n_counters)));
    WKE_TRY(dev_alloc(p, &p->d_ystage, 2 * p->total_elems));
    WKE_TRY(dev_alloc(p, &p->d_ksum, 2 * p->total_elems));
    WKE_TRY(dev_alloc(p, &p->d_mom, 7 * (size_t)batch));

    hipStream_t s = p->stream;
    HIP_TRY(hipMemcpyAsync(p->d_inst, p->inst.data(), sizeof(InstDev) * batch, hipMemcpyHostToDevice, s));
    std::vector<UnitPat> allpat;
    for (int i = 0; i < batch; ++i) allpat.insert(allpat.end(), p->pats[i].begin(), p->pats[i].end());
    HIP_TRY(hipMemcpyAsync(p->d_upat, allpat.data(), sizeof(UnitPat) * allpat.size(), hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(p->d_upat_off, pat_off.data(), sizeof(int) * batch, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemsetAsync(p->d_counters, 0, sizeof(unsigned int) * std::max(1, p->n_counters), s));
    for (auto& kv : p->tw_off)
        HIP_TRY(launch_twiddles(kv.first, p->d_tw64 + 2 * kv.second, p->d_tw32 + 2 * kv.second, s));
    for (int i = 0; i < batch; ++i)
        HIP_TRY(launch_tables(p->d_inst, p->inst[i], i, p->d_nodes, p->d_upat + pat_off[i], p->d_ph64, p->d_ph32,
                              p->d_uw64, p->d_uw32, s));
    // the host copies above read pageable buffers owned by this function
    HIP_TRY(hipStreamSynchronize(s));

    // shared slab fields: read back the quadrature, find the shifts that
    // agree on axes 1..d-1, and size the slab-field workspace
    std::vector<double> nodes(std::max<long long>(1, p->n_nodes));
    HIP_TRY(hipMemcpy(nodes.data(), p->d_nodes, sizeof(double) * p->n_nodes, hipMemcpyDeviceToHost));
    p->hrep.resize(batch);
    p->hid.resize(batch);
    p->frep.resize(batch);
    p->fid.resize(batch);
    p->rounds.resize(batch);
    p->flds.resize(batch);
    p->lidx.resize(batch);
    p->ig_r0.resize(batch);
    p->ig_r1.resize(batch);
    p->ig_f0.resize(batch);
    p->ig_nfl.resize(batch);
    p->fp_ng.assign(batch, 0);
    p->fp_ni.assign(batch, 0);
    long long n_hrep = 0, n_hid = 0, n_rounds = 0, n_kt = 0;
    for (int i = 0; i < batch; ++i) {
        InstDev& I = p->inst[i];
        group_shifts(I, nodes.data() + I.off_nodes, 1, &p->hrep[i], &p->hid[i]);
        group_shifts(I, nodes.data() + I.off_nodes, 0, &p->frep[i], &p->fid[i]);
        I.n_slab = (int)p->hrep[i].size();
        I.off_rounds = n_rounds;
        n_rounds += I.n_items;
        I.off_kt = n_kt;
        if (I.d == 2) n_kt += 2LL * I.n_slab * I.N;      // each row twice over
        I.off_G = p->n_G;
        p->n_G += (long long)I.n_slab * I.n_pts;
        I.off_hrep = n_hrep;
        n_hrep += I.n_slab;
        I.off_hid = n_hid;
        // per shift (and the zero shift); the real form's rounds hold up to
        // one more field each, and there are at most n_items rounds
        n_hid += I.n_shift + (long long)I.nyq_zero * (1 + I.n_items);
    }
    if (precision == WKE_F64) {
        double* b;
        WKE_TRY(dev_alloc(p, &b, 2 * p->n_G));
        p->d_G = b;
    } else {
        float* b;
        WKE_TRY(dev_alloc(p, &b, 2 * p->n_G));
        p->d_G = b;
    }
    std::vector<int> allrep, allhid(std::max<long long>(1, n_hid), 0);
    for (int i = 0; i < batch; ++i) {
        allrep.insert(allrep.end(), p->hrep[i].begin(), p->hrep[i].end());
        std::copy(p->hid[i].begin(), p->hid[i].end(), allhid.begin() + p->inst[i].off_hid);
    }
    WKE_TRY(dev_alloc(p, &p->d_hrep, allrep.size()));
    WKE_TRY(dev_alloc(p, &p->d_hid, allhid.size()));
    WKE_TRY(dev_alloc(p, &p->d_rounds, std::max<long long>(1, n_rounds)));
    WKE_TRY(dev_alloc(p, &p->d_flds, std::max<size_t>(1, allhid.size())));
    WKE_TRY(dev_alloc(p, &p->d_lidx, std::max<size_t>(1, allhid.size())));
    HIP_TRY(hipMemcpyAsync(p->d_hrep, allrep.data(), sizeof(int) * allrep.size(), hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(p->d_hid, allhid.data(), sizeof(int) * allhid.size(), hipMemcpyHostToDevice, s));
    // interpolation kernels of the 2D slab fields (the fused column pass)
    WKE_TRY(dev_alloc(p, &p->d_kt64, 2 * std::max<long long>(1, n_kt)));
    if (precision == WKE_F32) WKE_TRY(dev_alloc(p, &p->d_kt32, 2 * std::max<long long>(1, n_kt)));
    HIP_TRY(hipMemcpyAsync(p->d_inst, p->inst.data(), sizeof(InstDev) * batch, hipMemcpyHostToDevice, s));
    for (int i = 0; i < batch; ++i) {
        const InstDev& I = p->inst[i];
        if (I.d == 2 && I.off_kt + 2LL * I.n_slab * I.N > n_kt)
            return fail(WKE_ERR_INVALID, "internal: interpolation table of instance %d out of range", i);
        HIP_TRY(launch_ktab(p->d_inst, I, i, p->d_ph64, p->d_hrep, p->d_kt64, p->d_kt32, s));
    }

    // tasks, grouped by N
    for (Group& G : p->groups) {
        for (int i = 0; i < batch; ++i) {
            if (insts[i].N != G.N) continue;
            const InstDev& I = p->inst[i];
            Geometry g;
            geometry_of(precision, I.d, G.N, &g);
            // the real form needs the rows j0 = 0..N/2 only (the others are
            // their conjugates, read mirrored by the column pass)
            const int jend = p->nyq ? G.N / 2 + 1 : G.N;
            // the wider 3D workgroup where it brings the pass within one
            // workgroup per compute unit (measured at 3D N=32 double with 17
            // slab fields: 288 -> 192 workgroups, +5% per evaluation; with
            // many slab fields the narrower one is faster)
            const int rows = (jend + g.groups_a - 1) / g.groups_a;
            const int spt0 = g.shifts_per_task_a, spt1 = g.shifts_per_task_a_alt;
            const bool alt = spt1 > 0 && batch == 1 && rows * ((I.n_slab + spt0 - 1) / spt0) > 256 &&
                             rows * ((I.n_slab + spt1 - 1) / spt1) <= 256;
            if (alt) G.slab_alt = 1;
            const int spt = alt ? spt1 : spt0;
            for (int j0 = 0; j0 < jend; j0 += g.groups_a)
                for (int s0 = 0; s0 < I.n_slab; s0 += spt)
                    G.hA.push_back(TaskA{i, j0, s0, std::min(I.n_slab, s0 + spt)});
            const long long C = I.d == 2 ? I.N : (long long)I.N * I.N;
            for (int cb = 0; cb < (int)((C + g.groups_f - 1) / g.groups_f); ++cb)
                G.hF.push_back(TaskB{i, cb, 0, 0, 0, 0, 0, 0});
        }
        WKE_TRY(dev_alloc(p, &G.dA, G.hA.size()));
        size_t maxB = 0;
        for (int i = 0; i < batch; ++i)
            if (insts[i].N == G.N) {
                const InstDev& I = p->inst[i];
                const long long C = I.d == 2 ? I.N : (long long)I.N * I.N;
                const int gmin = std::min(fp_columns(I.d), g_slots_columns(precision, I.d, I.N));
                maxB += (size_t)((C + gmin - 1) / gmin) * p->max_ig[i];
            }
        WKE_TRY(dev_alloc(p, &G.dB, std::max<size_t>(1, maxB)));
        WKE_TRY(dev_alloc(p, &G.dF, G.hF.size()));
        HIP_TRY(hipMemcpyAsync(G.dA, G.hA.data(), sizeof(TaskA) * G.hA.size(), hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(G.dF, G.hF.data(), sizeof(TaskB) * G.hF.size(), hipMemcpyHostToDevice, s));
        G.colkind = fp_feasible(p, G) ? 1 : 0;
        if (p->nyq && !G.colkind)
            return fail(WKE_ERR_UNSUPPORTED, "the real form needs the field-parallel column pass (at most %d product "
                        "units per item and one item's fields in a workgroup)", FP_MAX_UNITS);
        size_t nwg = 0;
        for (int i = 0; i < batch; ++i)
            if (insts[i].N == G.N) nwg += (size_t)p->inst[i].n_cb * p->inst[i].n_ig;
        G.fp_wide = nwg < 256 ? 1 : 0;
        WKE_TRY(apply_split(p, G));      // column-pass tasks and rounds; uploads the descriptors
    }
    HIP_TRY(hipStreamSynchronize(s));
    return WKE_OK;
}

void drop_graph(wke_plan_s* p) {
    if (p->step_exec) (void)hipGraphExecDestroy(p->step_exec);
    p->step_exec = nullptr;
    p->graph_f = nullptr;
}

void free_plan(wke_plan_s* p) {
    if (!p) return;
    if (p->fine) free_plan(p->fine);
    if (!p->allocs.empty()) (void)hipStreamSynchronize(p->stream);
    drop_graph(p);
    if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
    for (void* q : p->allocs) (void)hipFree(q);
    delete p;
}

// Split instance i's quadrature sum over n workgroups per column block.
void set_split(wke_plan_s* p, int i, int n) {
    InstDev& I = p->inst[i];
    n = std::max(p->min_ig[i], std::min(n, p->max_ig[i]));
    I.items_per_ig = (I.n_items + n - 1) / n;
    I.n_ig = (I.n_items + I.items_per_ig - 1) / I.items_per_ig;
}

// Rounds of the field-parallel column pass for instance i under its current
// split: each item group's items are taken in order, and a round closes when
// the next item's new distinct fields would not fit the workgroup (cap lane
// groups) or its weights the weight buffer.
void build_rounds(wke_plan_s* p, int i, int cap) {
    const InstDev& I = p->inst[i];
    const int S = I.S_item, U = I.U_item;
    const std::vector<int>& fid = p->fid[i];
    const std::vector<int>& frep = p->frep[i];
    std::vector<RoundDesc>& rounds = p->rounds[i];
    std::vector<int2>& flds = p->flds[i];
    std::vector<int>& lidx = p->lidx[i];
    rounds.clear();
    flds.clear();
    lidx.assign(I.n_shift, 0);
    p->ig_r0[i].assign(I.n_ig, 0);
    p->ig_r1[i].assign(I.n_ig, 0);
    p->ig_f0[i].assign(I.n_ig, 0);
    p->ig_nfl[i].assign(I.n_ig, 0);
    int ng = 0, ni = 0;
    for (int ig = 0; ig < I.n_ig; ++ig) {
        const int it0 = ig * I.items_per_ig, it1 = std::min(I.n_items, it0 + I.items_per_ig);
        p->ig_r0[i][ig] = (int)rounds.size();
        p->ig_f0[i][ig] = (int)flds.size();
        for (int ia = it0; ia < it1;) {
            std::map<int, int> local;          // distinct field -> round-local index
            std::vector<int> order;
            if (I.nyq_zero) {                  // the real form's zero shift is local field 0 of every round
                local.emplace(fid[I.n_shift], 0);
                order.push_back(fid[I.n_shift]);
            }
            int ib = ia;
            while (ib < it1) {
                int fresh = 0;
                std::vector<int> seen;
                for (int f = 0; f < S; ++f) {
                    const int id = fid[ib * S + f];
                    if (!local.count(id) && std::find(seen.begin(), seen.end(), id) == seen.end()) {
                        seen.push_back(id);
                        ++fresh;
                    }
                }
                if (ib > ia && ((int)local.size() + fresh > cap || (ib - ia + 1) * U > FP_MAX_GROUPS)) break;
                for (int f = 0; f < S; ++f) {
                    const int id = fid[ib * S + f];
                    if (!local.count(id)) {
                        local.emplace(id, (int)order.size());
                        order.push_back(id);
                    }
                }
                ++ib;
            }
            rounds.push_back(RoundDesc{ia, ib, (int)flds.size(), (int)order.size()});
            for (int id : order) flds.push_back(make_int2(frep[id], p->hid[i][frep[id]]));
            for (int ls = ia * S; ls < ib * S; ++ls) lidx[ls] = local[fid[ls]];
            ng = std::max(ng, (int)order.size());
            ni = std::max(ni, ib - ia);
            ia = ib;
        }
        p->ig_r1[i][ig] = (int)rounds.size();
        p->ig_nfl[i][ig] = (int)flds.size() - p->ig_f0[i][ig];
    }
    p->fp_ng[i] = ng;
    p->fp_ni[i] = ni;
}

// Column-pass tasks and field-parallel rounds for the group's current
// splits, uploaded (waits for the plan's stream first).
wke_status apply_split(wke_plan_s* p, Group& G) {
    // the rounds are built whenever the field-parallel forms apply, so that
    // their launch shapes can be judged from any current form
    const int half = G.colkind == 1 && G.fp_half && fp_feasible(p, G, 1) ? 1 : 0;
    const int cap = fp_feasible(p, G) ? fp_field_cap(p, G.N, half) : 0;
    G.hB.clear();
    for (int i = 0; i < p->batch; ++i) {
        if (p->inst[i].N != G.N) continue;
        InstDev& I = p->inst[i];
        const long long C = I.d == 2 ? I.N : (long long)I.N * I.N;
        const int gb = G.colkind >= 1 ? fp_columns(I.d) : g_slots_columns(p->prec, I.d, I.N);
        I.n_cb = (int)((C + gb - 1) / gb);
        if (cap > 0) build_rounds(p, i, cap);
        for (int cb = 0; cb < I.n_cb; ++cb)
            for (int ig = 0; ig < I.n_ig; ++ig) {
                TaskB tb{i, cb, ig, 0, 0, 0, 0, 0};
                if (cap > 0 && G.colkind >= 1) {
                    tb.r0 = p->ig_r0[i][ig];
                    tb.r1 = p->ig_r1[i][ig];
                    tb.f0 = p->ig_f0[i][ig];
                    tb.nfl = p->ig_nfl[i][ig];
                }
                G.hB.push_back(tb);
            }
    }
    update_fp(p, G);
    HIP_TRY(hipStreamSynchronize(p->stream));
    HIP_TRY(hipMemcpy(p->d_inst, p->inst.data(), sizeof(InstDev) * p->batch, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(G.dB, G.hB.data(), sizeof(TaskB) * G.hB.size(), hipMemcpyHostToDevice));
    if (cap > 0) {
        for (int i = 0; i < p->batch; ++i) {
            if (p->inst[i].N != G.N) continue;
            const InstDev& I = p->inst[i];
            HIP_TRY(hipMemcpy(p->d_rounds + I.off_rounds, p->rounds[i].data(),
                              sizeof(RoundDesc) * p->rounds[i].size(), hipMemcpyHostToDevice));
            HIP_TRY(hipMemcpy(p->d_flds + I.off_hid, p->flds[i].data(), sizeof(int2) * p->flds[i].size(),
                              hipMemcpyHostToDevice));
            HIP_TRY(hipMemcpy(p->d_lidx + I.off_hid, p->lidx[i].data(), sizeof(int) * p->lidx[i].size(),
                              hipMemcpyHostToDevice));
        }
    }
    return WKE_OK;
}

const void* ph_ptr(const wke_plan_s* p) { return p->prec == WKE_F64 ? (const void*)p->d_ph64 : (const void*)p->d_ph32; }
const void* uw_ptr(const wke_plan_s* p) { return p->prec == WKE_F64 ? (const void*)p->d_uw64 : (const void*)p->d_uw32; }
const void* tw_ptr(const wke_plan_s* p) { return p->prec == WKE_F64 ? (const void*)p->d_tw64 : (const void*)p->d_tw32; }

wke_status run_colfwd(wke_plan_s* p, const double* f) {
    for (Group& G : p->groups) {
        // the fused column pass reads spec0 column-major
        ColFwdArgs a{p->d_inst, G.dF, f, p->d_spec0, tw_ptr(p), G.colkind == 2 ? 1 : 0};
        HIP_TRY(launch_colfwd(p->prec, p->d, G.N, a, (int)G.hF.size(), p->stream));
    }
    return WKE_OK;
}

hipError_t group_passA(wke_plan_s* p, Group& G, const LaunchEvents* ev = nullptr) {
    if (G.colkind == 2) return hipSuccess;       // the fused column pass builds its slab fields itself
    PassAArgs a{p->d_inst, G.dA, p->d_spec0, p->d_G, ph_ptr(p), p->d_hrep, tw_ptr(p), G.slab_alt};
    return launch_passA(p->prec, p->d, G.N, a, (int)G.hA.size(), p->stream, ev);
}

wke_status run_passA(wke_plan_s* p, const std::vector<LaunchEvents>* ev = nullptr) {
    size_t gi = 0;
    for (Group& G : p->groups) {
        HIP_TRY(group_passA(p, G, ev ? &(*ev)[gi] : nullptr));
        ++gi;
    }
    return WKE_OK;
}

PassBArgs passB_args(const wke_plan_s* p, const Group& G, int mode, int stage, const double* F0, double* out,
                     double* y, double dt) {
    PassBArgs a{};
    a.inst = p->d_inst;
    a.tasks = G.dB;
    a.G = p->d_G;
    a.hid = p->d_hid;
    a.ph = ph_ptr(p);
    a.rounds = p->d_rounds;
    a.flds = p->d_flds;
    a.lidx = p->d_lidx;
    a.spec0 = p->d_spec0;
    a.F0 = F0;
    a.out = out;
    a.y = y;
    a.ystage = p->d_ystage;
    a.ksum = p->d_ksum;
    a.uw = uw_ptr(p);
    a.upat = p->d_upat;
    a.upat_off = p->d_upat_off;
    a.part = p->d_part;
    a.counters = p->d_counters;
    a.tw = tw_ptr(p);
    a.mode = mode;
    a.stage = stage;
    a.dt = dt;
    a.fp_threads = G.colkind >= 1 ? G.fp_threads : 0;
    a.fp_lds = G.fp_lds;
    a.fp_fused = G.colkind == 2 ? 1 : 0;
    a.fp_nwp = G.fp_nwp;
    a.fp_off_h = G.fp_off_h;
    a.fp_off_ph = G.fp_off_ph;
    a.kt = p->prec == WKE_F64 ? (const void*)p->d_kt64 : (const void*)p->d_kt32;
    a.real = p->nyq;
    return a;
}

wke_status run_passB(wke_plan_s* p, int mode, int stage, const double* F0, double* out, double* y, double dt,
                     const std::vector<LaunchEvents>* ev = nullptr) {
    size_t gi = 0;
    for (Group& G : p->groups) {
        const PassBArgs a = passB_args(p, G, mode, stage, F0, out, y, dt);
        HIP_TRY(launch_passB(p->prec, p->d, G.N, a, (int)G.hB.size(), p->stream, ev ? &(*ev)[gi] : nullptr));
        ++gi;
    }
    return WKE_OK;
}

// ---------------------------------------------------------------------------
// Exact-Galerkin (de-aliased) plans.  The mode constraint l + m + n = j of
// eq. (KK1) holds without wrap-around when every transform of Alg. 1 is
// taken on 2N points instead of N (the remark on zero padding after the
// truncation in Section 3): the product of three series with modes in
// [-N/2, N/2-1] has modes in [-3N/2, 3N/2-3], and none of them wraps into
// [-N/2, N/2-1] modulo 2N.  So Q is the cyclic operator of the fine plan
// applied to the truncated series of f sampled on the fine grid, projected
// back onto the modes [-N/2, N/2-1] and sampled on the coarse grid.
// ---------------------------------------------------------------------------

wke_status build_galerkin(wke_plan_s* p, const wke_desc* insts, int batch, int precision) {
    for (int i = 0; i < batch; ++i) {
        const wke_desc& q = insts[i];
        if (q.d != 2 && q.d != 3) return fail(WKE_ERR_INVALID, "instance %d: d must be 2 or 3", i);
        if (q.N < 2 || (q.N & 1)) return fail(WKE_ERR_INVALID, "instance %d: N must be even and >= 2", i);
        if (!supported_N(q.d, 2 * q.N) || q.N % 4)
            return fail(WKE_ERR_UNSUPPORTED, "instance %d: the exact-Galerkin form runs on 2N = %d points, "
                        "which is not built for d = %d", i, 2 * q.N, q.d);
    }
    std::vector<wke_desc> fd(insts, insts + batch);
    for (wke_desc& q : fd) q.N *= 2;
    WKE_TRY(validate(fd.data(), batch, precision));
    p->fine = new (std::nothrow) wke_plan_s();
    if (!p->fine) return fail(WKE_ERR_NOMEM, "host allocation failed");
    p->fine->stream = p->stream;
    WKE_TRY(build_plan(p->fine, fd.data(), batch, precision));
    const wke_plan_s* F = p->fine;

    p->batch = batch;
    p->prec = precision;
    p->d = insts[0].d;
    p->desc.assign(insts, insts + batch);
    p->device = F->device;
    p->inst.resize(batch);
    long long off = 0;
    for (int i = 0; i < batch; ++i) {
        InstDev& I = p->inst[i];
        I = F->inst[i];             // quadrature as on the fine grid
        I.N = insts[i].N;
        I.h = 2.0 * I.L / I.N;
        long long np = 1;
        for (int a = 0; a < I.d; ++a) np *= I.N;
        I.n_pts = np;
        I.fwd_scale = 1.0 / (double)np;
        I.off_state = off;
        off += np;
    }
    p->total_elems = (size_t)off;
    const size_t nf = F->total_elems;
    WKE_TRY(dev_alloc(p, &p->d_inst, (size_t)batch));
    WKE_TRY(dev_alloc(p, &p->d_mom, 7 * (size_t)batch));
    WKE_TRY(dev_alloc(p, &p->d_ystage, 2 * p->total_elems));
    WKE_TRY(dev_alloc(p, &p->d_ksum, 2 * p->total_elems));
    WKE_TRY(dev_alloc(p, &p->d_fP, 2 * nf));
    WKE_TRY(dev_alloc(p, &p->d_QP, 2 * nf));
    WKE_TRY(dev_alloc(p, &p->d_t1, 2 * nf));
    WKE_TRY(dev_alloc(p, &p->d_t2, 2 * nf));
    WKE_TRY(dev_alloc(p, &p->d_ysP, 2 * nf));
    WKE_TRY(dev_alloc(p, &p->d_ksP, 2 * nf));
    WKE_TRY(dev_alloc(p, &p->d_fine_off, (size_t)batch));

    // kernels h_k = sum_{j=-N/2}^{N/2-1} e^{2 pi i j (2k+1) / 2N}, angles
    // reduced exactly modulo 2N before the sine and cosine
    std::vector<double> h;
    std::vector<int> h_off(batch);
    for (int i = 0; i < batch; ++i) {
        const int N = insts[i].N, P = 2 * N;
        h_off[i] = (int)(h.size() / 2);
        for (int k = 0; k < N; ++k) {
            double re = 0.0, im = 0.0;
            for (int j = -N / 2; j < N / 2; ++j) {
                const long long m = (((long long)j * (2 * k + 1)) % P + P) % P;
                const double ang = 2.0 * M_PI * (double)m / (double)P;
                re += std::cos(ang);
                im += std::sin(ang);
            }
            h.push_back(re);
            h.push_back(im);
        }
    }
    WKE_TRY(dev_alloc(p, &p->d_hres, h.size()));

    // descriptors: refining axes d-1..0 (f -> t1 (-> t2) -> fP), then
    // coarsening axes d-1..0 (QP -> t1 (-> t2) -> coarse output), then
    // projecting axes d-1..1 on the fine grid (QP -> t1 (-> t2))
    const int d = p->d;
    std::vector<ResampleDesc> rs;
    p->rs_launch.assign(3 * d - 1, ResampleLaunch{1, 1, 0});
    for (int dir = 0; dir < 3; ++dir) {
        for (int k = 0; k < (dir == 2 ? d - 1 : d); ++k) {
            const int a = d - 1 - k, pass = dir * d + k;
            for (int i = 0; i < batch; ++i) {
                const int N = insts[i].N, P = 2 * N;
                int ext[3];
                for (int b = 0; b < d; ++b) ext[b] = dir == 0 ? (b > a ? P : N) : (dir == 1 && b > a ? N : P);
                ResampleDesc D{};
                D.m_in = ext[a];
                D.m_out = dir == 0 || dir == 2 ? P : N;
                ext[a] = D.m_out;
                D.inner = 1;
                for (int b = a + 1; b < d; ++b) D.inner *= ext[b];
                D.n_out = 1;
                for (int b = 0; b < d; ++b) D.n_out *= ext[b];
                D.N = N;
                D.h_off = h_off[i];
                // the coarse end of each chain uses the coarse packing
                D.in_off = dir == 0 && k == 0 ? p->inst[i].off_state : F->inst[i].off_state;
                // (projections stay on the fine grid)
                D.out_off = dir == 1 && k == d - 1 ? p->inst[i].off_state : F->inst[i].off_state;
                rs.push_back(D);
            }
            // N work items per line (one per odd fine or coarse point), about
            // one per thread: lt = 256 / N lines per workgroup
            ResampleLaunch& g = p->rs_launch[pass];
            int n_max = 1;
            for (int i = 0; i < batch; ++i) n_max = std::max(n_max, insts[i].N);
            g.lt = std::max(1, 256 / n_max);
            long long blocks = 1;
            size_t lds = 0;
            for (int i = 0; i < batch; ++i) {
                const ResampleDesc& D = rs[pass * batch + i];
                blocks = std::max(blocks, (D.n_out / D.m_out + g.lt - 1) / g.lt);
                lds = std::max(lds, sizeof(double) * 2 * (size_t)(2 * D.N + (long long)g.lt * D.m_in));
            }
            if (blocks > (1LL << 30) || lds > 64 * 1024)
                return fail(WKE_ERR_UNSUPPORTED, "resampling launch out of range");
            g.blocks = (int)blocks;
            g.lds = (unsigned)lds;
        }
    }
    WKE_TRY(dev_alloc(p, &p->d_rs, rs.size()));
    hipStream_t s = p->stream;
    HIP_TRY(hipMemcpyAsync(p->d_inst, p->inst.data(), sizeof(InstDev) * batch, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(p->d_hres, h.data(), sizeof(double) * h.size(), hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(p->d_rs, rs.data(), sizeof(ResampleDesc) * rs.size(), hipMemcpyHostToDevice, s));
    std::vector<long long> fo(batch);
    for (int i = 0; i < batch; ++i) fo[i] = F->inst[i].off_state;
    HIP_TRY(hipMemcpyAsync(p->d_fine_off, fo.data(), sizeof(long long) * batch, hipMemcpyHostToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));   // the host vectors go out of scope
    return WKE_OK;
}

// The buffers of resampling launch k of a chain (dir 0 refining, 1 coarsening).
void chain_buffers(const wke_plan_s* p, int dir, int k, const double* first, double* last, const double** in,
                   double** out) {
    const int d = p->d;
    double* mid[2] = {p->d_t1, p->d_t2};
    *in = k == 0 ? first : mid[k - 1];
    *out = k == d - 1 ? last : mid[k];
}

// f (coarse) -> the truncated series of f on the fine grid, in d_fP.
wke_status refine(wke_plan_s* p, const double* f) {
    for (int k = 0; k < p->d; ++k) {
        const double* in;
        double* out;
        chain_buffers(p, 0, k, f, p->d_fP, &in, &out);
        HIP_TRY(launch_resample(RS_REFINE, p->d_rs + (size_t)k * p->batch, p->batch, p->rs_launch[k], p->d_hres, in,
                                out, p->stream));
    }
    return WKE_OK;
}

// d_QP -> its projection on the coarse grid, stored in Q.
wke_status coarsen(wke_plan_s* p, double* Q) {
    for (int k = 0; k < p->d; ++k) {
        const double* in;
        double* out;
        chain_buffers(p, 1, k, p->d_QP, Q, &in, &out);
        const int pass = p->d + k;
        HIP_TRY(launch_resample(RS_COARSEN, p->d_rs + (size_t)pass * p->batch, p->batch, p->rs_launch[pass],
                                p->d_hres, in, out, p->stream));
    }
    return WKE_OK;
}

// One exact-Galerkin RK4 stage kept on the fine grid: the fine-grid state
// (d_fP) and stage buffers hold functions of the coarse modes only, so f_N of
// the stage state is the fine-grid state itself.  The operator's result is
// projected onto the coarse modes, along axes d-1..1 by resampling launches
// and along axis 0 inside k_colrk, which also takes the stage update and the
// next axis-0 transform.
wke_status galerkin_stage(wke_plan_s* p, int stage, double dt) {
    wke_plan_s* F = p->fine;
    WKE_TRY(run_passA(F));
    WKE_TRY(run_passB(F, MODE_EVAL, 0, stage == 0 ? p->d_fP : p->d_ysP, p->d_QP, nullptr, 0.0));
    const double* q = p->d_QP;
    double* mid[2] = {p->d_t1, p->d_t2};
    for (int k = 0; k < p->d - 1; ++k) {
        const int pass = 2 * p->d + k;
        HIP_TRY(launch_resample(RS_PROJECT, p->d_rs + (size_t)pass * p->batch, p->batch, p->rs_launch[pass],
                                p->d_hres, q, mid[k], p->stream));
        q = mid[k];
    }
    for (Group& G : F->groups) {
        ColRkArgs a{};
        a.inst = F->d_inst;
        a.tasks = G.dF;
        a.q = q;
        a.y = p->d_fP;
        a.ys = p->d_ysP;
        a.ks = p->d_ksP;
        a.spec0 = F->d_spec0;
        a.tw64 = F->d_tw64;
        a.tw = tw_ptr(F);
        a.spec_trans = G.colkind == 2 ? 1 : 0;
        a.stage = stage;
        a.dt = dt;
        HIP_TRY(launch_colrk(F->prec, F->d, G.N, a, (int)G.hF.size(), p->stream));
    }
    return WKE_OK;
}

wke_status galerkin_step(wke_plan_s* p, double* f, double dt, int nsteps) {
    WKE_TRY(refine(p, f));
    WKE_TRY(run_colfwd(p->fine, p->d_fP));
    for (int n = 0; n < nsteps; ++n)
        for (int st = 0; st < 4; ++st) WKE_TRY(galerkin_stage(p, st, dt));
    int n_max = 1;
    for (const wke_desc& q : p->desc) n_max = std::max(n_max, q.N);
    HIP_TRY(launch_decimate(p->d_rs + (size_t)(2 * p->d - 1) * p->batch, p->d_fine_off, p->batch, p->d, n_max,
                            p->d_fP, f, p->stream));
    return WKE_OK;
}

wke_status galerkin_eval(wke_plan_s* p, const double* f, double* Q) {
    wke_plan_s* F = p->fine;
    WKE_TRY(refine(p, f));
    WKE_TRY(run_colfwd(F, p->d_fP));
    WKE_TRY(run_passA(F));
    WKE_TRY(run_passB(F, MODE_EVAL, 0, p->d_fP, p->d_QP, nullptr, 0.0));
    return coarsen(p, Q);
}

}  // namespace

extern "C" {

const char* wke_status_string(wke_status s) {
    switch (s) {
        case WKE_OK: return "ok";
        case WKE_ERR_INVALID: return "invalid argument";
        case WKE_ERR_UNSUPPORTED: return "unsupported configuration";
        case WKE_ERR_HIP: return "HIP runtime error";
        case WKE_ERR_NOMEM: return "out of device memory";
        case WKE_ERR_NONFINITE: return "non-finite value";
    }
    return "unknown status";
}

const char* wke_last_error(void) { return g_last_error.c_str(); }

void wke_test_fail_allocations(int after) { g_alloc_budget.store(after < 0 ? -1 : (long)after); }

wke_status wke_plan_create(wke_plan_t* out, const wke_desc* insts, int batch, int precision, void* stream) {
    if (!out) return fail(WKE_ERR_INVALID, "out is NULL");
    *out = nullptr;
    WKE_TRY(validate(insts, batch, precision));
    wke_plan_s* p = new (std::nothrow) wke_plan_s();
    if (!p) return fail(WKE_ERR_NOMEM, "host allocation failed");
    p->stream = static_cast<hipStream_t>(stream);
    wke_status st = build_plan(p, insts, batch, precision);
    if (st != WKE_OK) {
        free_plan(p);
        return st;
    }
    *out = p;
    g_last_error.clear();
    return WKE_OK;
}

}  // extern "C"

namespace {

// Arguments and workspace sizes (doubles, in the order rk, uk, S, phi, F, Qh)
// of the exact-weight reference system; validates the descriptor.
wke_status exact_setup(const wke_desc* desc, int n_radial, const double* f, double* Q, ExactArgs* a,
                       size_t sizes[6]) {
    if (!desc || !f || !Q) return fail(WKE_ERR_INVALID, "NULL argument");
    if ((const double*)Q == f) return fail(WKE_ERR_INVALID, "Q must not alias f");
    const int d = desc->d, N = desc->N;
    if (d != 2 && d != 3) return fail(WKE_ERR_INVALID, "d must be 2 or 3");
    if (N < 2 || (N & 1)) return fail(WKE_ERR_INVALID, "N must be even and >= 2");
    if (!(desc->L > 0.0) || !std::isfinite(desc->L) || !std::isfinite(desc->R))
        return fail(WKE_ERR_INVALID, "L must be positive and R finite");
    if (n_radial < 1 || n_radial > 4096) return fail(WKE_ERR_INVALID, "n_radial must be in 1..4096");
    long long n = 1;
    for (int k = 0; k < d; ++k) n *= N;
    if (n > 1024) return fail(WKE_ERR_UNSUPPORTED, "the O(N^(3d)) reference system takes N^d <= 1024");
    const double R = desc->R > 0 ? desc->R : 4.0 * desc->L / (3.0 + std::sqrt(2.0));
    if (R > 2.0 * desc->L) return fail(WKE_ERR_INVALID, "R must not exceed 2L");
    *a = ExactArgs{};
    a->d = d;
    a->N = N;
    a->nr = n_radial;
    a->A = 4 * d * N * N;
    a->B = d * (N - 1) * (N - 1);
    a->L = desc->L;
    a->R = R;
    a->f = f;
    a->Q = Q;
    sizes[0] = sizes[1] = (size_t)n_radial;
    sizes[2] = (size_t)(a->A + 1) * n_radial;
    sizes[3] = (size_t)(a->A + 1) * (a->B + 1);
    sizes[4] = sizes[5] = 2 * (size_t)n;
    return WKE_OK;
}

double** exact_ptr(ExactArgs* a, int i) {
    double** ptrs[6] = {&a->rk, &a->uk, &a->S, &a->phi, &a->F, &a->Qh};
    return ptrs[i];
}

}  // namespace

extern "C" {

wke_status wke_exact_system(const wke_desc* desc, int n_radial, const double* f, double* Q, void* stream) {
    ExactArgs a;
    size_t sizes[6];
    WKE_TRY(exact_setup(desc, n_radial, f, Q, &a, sizes));
    std::vector<void*> mem;
    wke_status st = WKE_OK;
    for (int i = 0; i < 6 && st == WKE_OK; ++i) {
        void* q = nullptr;
        if (alloc_device(&q, sizes[i] * sizeof(double)) != hipSuccess) {
            st = fail(WKE_ERR_NOMEM, "device allocation of %zu bytes failed", sizes[i] * sizeof(double));
        } else {
            mem.push_back(q);
            *exact_ptr(&a, i) = static_cast<double*>(q);
        }
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (st == WKE_OK) {
        hipError_t e = launch_exact(a, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) st = fail(WKE_ERR_HIP, "exact system: %s", hipGetErrorString(e));
    }
    for (void* q : mem) (void)hipFree(q);
    return st;
}

wke_status wke_exact_system_noalloc(const wke_desc* desc, int n_radial, const double* f, double* Q, void* stream) {
    ExactArgs a;
    size_t sizes[6];
    WKE_TRY(exact_setup(desc, n_radial, f, Q, &a, sizes));
    // each part starts on a 256-byte boundary of the static workspace
    size_t off[6], total = 0;
    for (int i = 0; i < 6; ++i) {
        off[i] = total;
        total += (sizes[i] + 31) / 32 * 32;
    }
    if (total > EXACT_SCRATCH_DOUBLES)
        return fail(WKE_ERR_UNSUPPORTED, "the allocation-free reference system needs %zu bytes of workspace for "
                    "d = %d, N = %d, %d radial points; its static workspace holds %zu", total * sizeof(double),
                    desc->d, desc->N, n_radial, EXACT_SCRATCH_DOUBLES * sizeof(double));
    double* base = nullptr;
    HIP_TRY(exact_scratch(&base));
    for (int i = 0; i < 6; ++i) *exact_ptr(&a, i) = base + off[i];
    HIP_TRY(launch_exact(a, static_cast<hipStream_t>(stream)));
    return WKE_OK;
}

wke_status wke_plan_create_real(wke_plan_t* out, const wke_desc* insts, int batch, int precision, void* stream) {
    if (!out) return fail(WKE_ERR_INVALID, "out is NULL");
    *out = nullptr;
    WKE_TRY(validate(insts, batch, precision));
    wke_plan_s* p = new (std::nothrow) wke_plan_s();
    if (!p) return fail(WKE_ERR_NOMEM, "host allocation failed");
    p->stream = static_cast<hipStream_t>(stream);
    p->nyq = 1;
    wke_status st = build_plan(p, insts, batch, precision);
    if (st != WKE_OK) {
        free_plan(p);
        return st;
    }
    *out = p;
    g_last_error.clear();
    return WKE_OK;
}

wke_status wke_plan_create_galerkin(wke_plan_t* out, const wke_desc* insts, int batch, int precision,
                                    void* stream) {
    if (!out) return fail(WKE_ERR_INVALID, "out is NULL");
    *out = nullptr;
    if (!insts || batch < 1) return fail(WKE_ERR_INVALID, "need at least one instance");
    if (precision != WKE_F64 && precision != WKE_F32) return fail(WKE_ERR_INVALID, "precision must be WKE_F64 or WKE_F32");
    wke_plan_s* p = new (std::nothrow) wke_plan_s();
    if (!p) return fail(WKE_ERR_NOMEM, "host allocation failed");
    p->stream = static_cast<hipStream_t>(stream);
    wke_status st = build_galerkin(p, insts, batch, precision);
    if (st != WKE_OK) {
        free_plan(p);
        return st;
    }
    *out = p;
    g_last_error.clear();
    return WKE_OK;
}

void wke_plan_destroy(wke_plan_t plan) { free_plan(plan); }

size_t wke_offset(wke_plan_t p, int i) {
    if (!p || i < 0 || i >= p->batch) return 0;
    return (size_t)p->inst[i].off_state;
}

size_t wke_total_elems(wke_plan_t p) { return p ? p->total_elems : 0; }

wke_status wke_eval_Q(wke_plan_t p, const double* f, double* Q) {
    if (!p || !f || !Q) return fail(WKE_ERR_INVALID, "NULL plan or pointer");
    if ((const double*)Q == f) return fail(WKE_ERR_INVALID, "Q must not alias f");
    if (p->fine) return galerkin_eval(p, f, Q);
    WKE_TRY(run_colfwd(p, f));
    WKE_TRY(run_passA(p));
    WKE_TRY(run_passB(p, MODE_EVAL, 0, f, Q, nullptr, 0.0));
    return WKE_OK;
}

wke_status wke_eval_Q_hat(wke_plan_t p, const double* f, double* Qhat) {
    if (!p || !f || !Qhat) return fail(WKE_ERR_INVALID, "NULL plan or pointer");
    for (int i = 0; i < p->batch; ++i) {
        const int N = p->desc[i].N;
        if (N != 8 && N != 16 && N != 32 && N != 48 && N != 64 && N != 96 && N != 128)
            return fail(WKE_ERR_UNSUPPORTED, "no Fourier-coefficient transform for N = %d", N);
    }
    WKE_TRY(wke_eval_Q(p, f, Qhat));
    for (int i = 0; i < p->batch; ++i)
        HIP_TRY(launch_spectrum(p->desc[i].d, p->desc[i].N, Qhat + 2 * (long long)wke_offset(p, i), p->stream));
    return WKE_OK;
}

namespace {

wke_status enqueue_rk_step(wke_plan_s* p, double* f, double dt) {
    for (int st = 0; st < 4; ++st) {
        WKE_TRY(run_passA(p));
        WKE_TRY(run_passB(p, MODE_RK, st, st == 0 ? f : p->d_ystage, nullptr, f, dt));
    }
    return WKE_OK;
}

// Capture one RK4 step for (f, dt) on the plan's private capture stream.
wke_status capture_step(wke_plan_s* p, double* f, double dt) {
    drop_graph(p);
    if (!p->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking));
    hipStream_t user = p->stream;
    p->stream = p->cap_stream;
    hipError_t e = hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal);
    wke_status st = e == hipSuccess ? enqueue_rk_step(p, f, dt) : fail(WKE_ERR_HIP, "capture: %s", hipGetErrorString(e));
    hipGraph_t graph = nullptr;
    hipError_t e2 = hipStreamEndCapture(p->cap_stream, &graph);
    p->stream = user;
    if (st != WKE_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return st;
    }
    if (e2 != hipSuccess) return fail(WKE_ERR_HIP, "end capture: %s", hipGetErrorString(e2));
    e = hipGraphInstantiate(&p->step_exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
        p->step_exec = nullptr;
        return fail(WKE_ERR_HIP, "graph instantiate: %s", hipGetErrorString(e));
    }
    p->graph_f = f;
    p->graph_dt = dt;
    return WKE_OK;
}

}  // namespace

wke_status wke_step(wke_plan_t p, double* f, double dt, int nsteps) {
    if (!p || !f) return fail(WKE_ERR_INVALID, "NULL plan or pointer");
    if (nsteps < 0 || !std::isfinite(dt)) return fail(WKE_ERR_INVALID, "bad dt or nsteps");
    if (nsteps == 0) return WKE_OK;
    if (p->fine) return galerkin_step(p, f, dt, nsteps);
    WKE_TRY(run_colfwd(p, f));
    if (p->use_graphs) {
        if (!p->step_exec || p->graph_f != f || p->graph_dt != dt) WKE_TRY(capture_step(p, f, dt));
        for (int n = 0; n < nsteps; ++n) HIP_TRY(hipGraphLaunch(p->step_exec, p->stream));
        return WKE_OK;
    }
    for (int n = 0; n < nsteps; ++n) WKE_TRY(enqueue_rk_step(p, f, dt));
    return WKE_OK;
}

wke_status wke_set_graphs(wke_plan_t p, int enable) {
    if (!p) return fail(WKE_ERR_INVALID, "NULL plan");
    if (p->fine && enable) return fail(WKE_ERR_UNSUPPORTED, "graph replay is not built for exact-Galerkin plans");
    p->use_graphs = enable != 0;
    if (!p->use_graphs) drop_graph(p);
    return WKE_OK;
}

wke_status wke_moments(wke_plan_t p, const double* f, double* out) {
    if (!p || !f || !out) return fail(WKE_ERR_INVALID, "NULL plan or pointer");
    HIP_TRY(launch_moments(p->d_inst, p->batch, f, p->d_mom, p->stream));
    std::vector<double> h(7 * (size_t)p->batch);
    HIP_TRY(hipMemcpyAsync(h.data(), p->d_mom, sizeof(double) * h.size(), hipMemcpyDeviceToHost, p->stream));
    HIP_TRY(hipStreamSynchronize(p->stream));
    bool bad = false;
    for (int i = 0; i < p->batch; ++i) {
        for (int q = 0; q < 6; ++q) {
            out[6 * i + q] = h[7 * i + q];
            if (!std::isfinite(h[7 * i + q])) bad = true;
        }
        if (h[7 * i + 6] != 0.0) bad = true;
    }
    if (bad) return fail(WKE_ERR_NONFINITE, "state holds NaN or infinite values");
    return WKE_OK;
}

wke_status wke_get_nodes(wke_plan_t p, int i, double* r, double* wr, double* qh, double* ws, double* sg,
                         double* wsig) {
    if (!p || i < 0 || i >= p->batch) return fail(WKE_ERR_INVALID, "bad plan or instance");
    if (!r || !wr || !qh || !ws || !sg || !wsig) return fail(WKE_ERR_INVALID, "NULL output");
    if (p->fine) return wke_get_nodes(p->fine, i, r, wr, qh, ws, sg, wsig);
    const InstDev& I = p->inst[i];
    const size_t n = 2 * I.Nr + (size_t)(I.d + 1) * (I.Ns + I.Nsig);
    std::vector<double> h(n);
    HIP_TRY(hipMemcpyAsync(h.data(), p->d_nodes + I.off_nodes, sizeof(double) * n, hipMemcpyDeviceToHost, p->stream));
    HIP_TRY(hipStreamSynchronize(p->stream));
    size_t o = 0;
    std::memcpy(r, &h[o], sizeof(double) * I.Nr); o += I.Nr;
    std::memcpy(wr, &h[o], sizeof(double) * I.Nr); o += I.Nr;
    std::memcpy(qh, &h[o], sizeof(double) * I.Ns * I.d); o += (size_t)I.Ns * I.d;
    std::memcpy(ws, &h[o], sizeof(double) * I.Ns); o += I.Ns;
    std::memcpy(sg, &h[o], sizeof(double) * I.Nsig * I.d); o += (size_t)I.Nsig * I.d;
    std::memcpy(wsig, &h[o], sizeof(double) * I.Nsig);
    return WKE_OK;
}

wke_status wke_time_kernels(wke_plan_t p, const double* f, double* Q, int reps, double* us_out) {
    if (!p || !f || !Q || !us_out || reps < 1) return fail(WKE_ERR_INVALID, "bad arguments");
    if ((const double*)Q == f) return fail(WKE_ERR_INVALID, "Q must not alias f");
    if (p->fine) {
        WKE_TRY(refine(p, f));
        return wke_time_kernels(p->fine, p->d_fP, p->d_QP, reps, us_out);
    }
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    wke_status st = WKE_OK;
    // kernel k: 0 column forward, 1 slab pass, 2 column pass (Q form),
    // 3 column pass (RK4 stage form, stage 1, on the plan's scratch state)
    auto launch = [&](int k) -> wke_status {
        if (k == 0) return run_colfwd(p, f);
        if (k == 1) return run_passA(p);
        if (k == 2) return run_passB(p, MODE_EVAL, 0, f, Q, nullptr, 0.0);
        return run_passB(p, MODE_RK, 1, f, nullptr, const_cast<double*>(f), 0.0);
    };
    for (int k = 0; k < 4 && st == WKE_OK; ++k) {
        if (k == 3) st = run_colfwd(p, f);   // spec0 and G back to f's before the RK form
        if (st == WKE_OK && k == 3) st = run_passA(p);
        // one untimed launch so every kernel sees its real inputs
        if (st == WKE_OK) st = launch(k);
        if (st != WKE_OK) break;
        if (hipEventRecord(e0, p->stream) != hipSuccess) { st = fail(WKE_ERR_HIP, "event record"); break; }
        for (int r = 0; r < reps && st == WKE_OK; ++r) st = launch(k);
        if (st != WKE_OK) break;
        if (hipEventRecord(e1, p->stream) != hipSuccess) { st = fail(WKE_ERR_HIP, "event record"); break; }
        if (hipEventSynchronize(e1) != hipSuccess) { st = fail(WKE_ERR_HIP, "event sync"); break; }
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) { st = fail(WKE_ERR_HIP, "elapsed time"); break; }
        us_out[k] = 1000.0 * ms / reps;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return st;
}

wke_status wke_plan_tune(wke_plan_t p, const double* f, double* Q, int reps, double* us_out) {
    if (!p || !f || !Q || reps < 1) return fail(WKE_ERR_INVALID, "bad arguments");
    drop_graph(p);    // the captured launches carry the old work split
    if ((const double*)Q == f) return fail(WKE_ERR_INVALID, "Q must not alias f");
    if (p->fine) {
        WKE_TRY(refine(p, f));
        return wke_plan_tune(p->fine, p->d_fP, p->d_QP, reps, us_out);
    }
    WKE_TRY(run_colfwd(p, f));
    WKE_TRY(run_passA(p));
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    wke_status st = WKE_OK;
    int gi = 0;
    for (Group& G : p->groups) {
        int cap = 1;
        for (int i = 0; i < p->batch; ++i)
            if (p->inst[i].N == G.N) cap = std::max(cap, p->max_ig[i]);
        std::vector<int> splits;
        for (int n = 1; n < cap; n *= 2) splits.push_back(n);
        splits.push_back(cap);
        // 0 item slots; 1, 2 field-parallel narrow, wide; 3, 4 fused narrow,
        // wide; 5, 6 field-parallel narrow, wide in half-width rounds.
        // Each candidate is timed as slab pass + column pass (the fused form
        // has no slab pass), on whatever spectrum layout is in place: only
        // the time matters here.
        std::vector<int> kinds;
        if (!p->nyq) kinds.push_back(0);      // the real form has no item-slot kernel
        if (fp_feasible(p, G)) {
            kinds.push_back(1);
            kinds.push_back(2);
            if (fused_width_ok(p, G, 0)) kinds.push_back(3);
            if (fused_width_ok(p, G, 1)) kinds.push_back(4);
            if (fp_feasible(p, G, 1)) {
                kinds.push_back(5);
                kinds.push_back(6);
            }
        }
        double best_us = 1e300;
        int best = splits[0], best_kind = kinds.empty() ? 0 : kinds[0];
        std::map<int, int> ng_full;     // split -> most fields in a round at full width
        for (int kind : kinds) {
            for (int n : splits) {
                for (int i = 0; i < p->batch; ++i)
                    if (p->inst[i].N == G.N) set_split(p, i, n);
                // half rounds that would hold the same fields as full ones
                // are the same launch: not timed again
                if (kind >= 5 && ng_full.count(n) && ng_full[n] <= fp_field_cap(p, G.N, 1)) continue;
                G.colkind = kind == 0 ? 0 : (kind == 3 || kind == 4 ? 2 : 1);
                G.fp_wide = kind == 2 || kind == 4 || kind == 6 ? 1 : 0;
                G.fp_half = kind >= 5 ? 1 : 0;
                if ((st = apply_split(p, G)) != WKE_OK) break;
                if (kind == 1) {
                    int ng = 0;
                    for (int i = 0; i < p->batch; ++i)
                        if (p->inst[i].N == G.N) ng = std::max(ng, p->fp_ng[i]);
                    ng_full[n] = ng;
                }
                // the RK4 stage form, as the time-stepping pipeline runs it
                // (stage 1 reads f as the base state and writes only the
                // plan's stage buffers and spectrum)
                const PassBArgs a = passB_args(p, G, MODE_RK, 1, f, nullptr, const_cast<double*>(f), 0.0);
                hipError_t e = group_passA(p, G);                                                // warm
                if (e == hipSuccess) e = launch_passB(p->prec, p->d, G.N, a, (int)G.hB.size(), p->stream);
                if (e == hipSuccess) e = hipEventRecord(e0, p->stream);
                for (int r = 0; r < reps && e == hipSuccess; ++r) {
                    e = group_passA(p, G);
                    if (e == hipSuccess) e = launch_passB(p->prec, p->d, G.N, a, (int)G.hB.size(), p->stream);
                }
                if (e == hipSuccess) e = hipEventRecord(e1, p->stream);
                if (e == hipSuccess) e = hipEventSynchronize(e1);
                float ms = 0.f;
                if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
                if (e != hipSuccess) { st = fail(WKE_ERR_HIP, "tuning launch failed: %s", hipGetErrorString(e)); break; }
                const double us = 1000.0 * ms / reps;
                if (us < best_us) { best_us = us; best = n; best_kind = kind; }
            }
            if (st != WKE_OK) break;
        }
        if (st != WKE_OK) break;
        for (int i = 0; i < p->batch; ++i)
            if (p->inst[i].N == G.N) set_split(p, i, best);
        G.colkind = best_kind == 0 ? 0 : (best_kind == 3 || best_kind == 4 ? 2 : 1);
        G.fp_wide = best_kind == 2 || best_kind == 4 || best_kind == 6 ? 1 : 0;
        G.fp_half = best_kind >= 5 ? 1 : 0;
        if ((st = apply_split(p, G)) != WKE_OK) break;
        if (us_out) {
            us_out[3 * gi] = G.colkind == 1 && G.fp_half ? WKE_COLUMN_FIELDS_HALF : G.colkind;
            us_out[3 * gi + 1] = best;
            us_out[3 * gi + 2] = best_us;
        }
        ++gi;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return st;
}

wke_status wke_plan_set_split(wke_plan_t p, int n) {
    if (!p || n < 1) return fail(WKE_ERR_INVALID, "bad arguments");
    if (p->fine) return wke_plan_set_split(p->fine, n);
    drop_graph(p);
    for (Group& G : p->groups) {
        for (int i = 0; i < p->batch; ++i)
            if (p->inst[i].N == G.N) set_split(p, i, n);
        WKE_TRY(apply_split(p, G));
    }
    return WKE_OK;
}

wke_status wke_plan_set_column_kernel(wke_plan_t p, int kind) {
    if (!p || (kind != WKE_COLUMN_SLOTS && kind != WKE_COLUMN_FIELDS && kind != WKE_COLUMN_FUSED &&
               kind != WKE_COLUMN_FIELDS_HALF))
        return fail(WKE_ERR_INVALID, "bad arguments");
    if (p->fine) return wke_plan_set_column_kernel(p->fine, kind);
    if (p->nyq && kind == WKE_COLUMN_SLOTS)
        return fail(WKE_ERR_UNSUPPORTED, "the real form has no item-slot column pass");
    if (kind == WKE_COLUMN_FIELDS || kind == WKE_COLUMN_FIELDS_HALF)
        for (const Group& G : p->groups)
            if (!fp_feasible(p, G, kind == WKE_COLUMN_FIELDS_HALF ? 1 : 0))
                return fail(WKE_ERR_UNSUPPORTED, "the field-parallel column pass needs at most %d product "
                            "units per item and one item's fields in a workgroup", FP_MAX_UNITS);
    if (kind == WKE_COLUMN_FUSED)
        for (Group& G : p->groups)
            if (!fused_feasible(p, G))
                return fail(WKE_ERR_UNSUPPORTED, "the fused column pass needs d = 2, the field-parallel form "
                            "and at most %d slab fields", FUSED_MAX_SLAB);
    drop_graph(p);
    HIP_TRY(hipStreamSynchronize(p->stream));
    for (Group& G : p->groups) {
        if (kind == WKE_COLUMN_FUSED) G.fp_wide = fused_width_ok(p, G, 1) ? 1 : 0;
        G.fp_half = kind == WKE_COLUMN_FIELDS_HALF ? 1 : 0;
        G.colkind = kind == WKE_COLUMN_FIELDS_HALF ? WKE_COLUMN_FIELDS : kind;
        WKE_TRY(apply_split(p, G));
    }
    return WKE_OK;
}

wke_status wke_field_counts(wke_plan_t p, int i, int* counts) {
    if (!p || !counts || i < 0 || i >= p->batch) return fail(WKE_ERR_INVALID, "bad arguments");
    if (p->fine) return wke_field_counts(p->fine, i, counts);
    counts[0] = p->inst[i].n_shift;
    counts[1] = p->inst[i].n_slab;
    counts[2] = (int)p->frep[i].size();
    return WKE_OK;
}

wke_status wke_work_model(wke_plan_t p, double* flops_out, double* bytes_out) {
    if (!p) return fail(WKE_ERR_INVALID, "NULL plan");
    if (p->fine) return wke_work_model(p->fine, flops_out, bytes_out);
    const double sz = p->prec == WKE_F64 ? 16.0 : 8.0;
    double f0 = 0, f1 = 0, f2 = 0, b0 = 0, b1 = 0, b2 = 0;
    for (int i = 0; i < p->batch; ++i) {
        const InstDev& I = p->inst[i];
        // transforms of the column pass: one per shift (item slots) or one
        // per distinct shift vector (field-parallel form)
        int colkind = 0;
        for (const Group& G : p->groups)
            if (G.N == I.N) colkind = G.colkind;
        double ncol = colkind >= 1 ? (double)p->frep[i].size() : (double)I.n_shift;
        if (I.nyq_zero) ncol = std::ceil(0.5 * ncol);      // two real fields per transform
        const double n = (double)I.n_pts;
        const double lgN = std::log2((double)I.N);
        const double lgR = (I.d - 1) * lgN;                    // log2 of the slab size
        f0 += 5.0 * n * lgN;                                   // axis-0 forward transform
        f2 += ncol * (5.0 * n * lgN + 6.0 * n)                 // axis-0 phase multiply + inverse
              + n * (I.nyq_zero ? 2.0 * I.n_items + 7.0 * I.n_unit      // real products
                                : 8.0 * I.n_items + 26.0 * I.n_unit);    // products and weighted sums
        b0 += n * (16.0 + sz);                                 // read f, write spec0
        b2 += n * (16.0 + 16.0) + ncol * I.N * sz;             // F0, Q, axis-0 phases
        if (colkind == 2) {
            // fused: every column interpolates its slab fields from spec0
            // (n_slab N complex multiply-adds per point), reading spec0 once
            f2 += 8.0 * n * I.N * I.n_slab;
            b2 += n * sz;
        } else {
            f1 += 5.0 * n * lgR                                // rest-axis forward transform
                  + I.n_slab * (5.0 * n * lgR + 6.0 * n);      // phase multiply + inverse, per slab field
            b1 += n * sz * (1.0 + I.n_slab) + (double)I.n_slab * (I.d - 1) * I.N * sz;   // spec0, slab fields, phases
            b2 += n * sz * I.n_slab;                           // slab fields (each read once)
        }
        if (I.n_ig > 1) b2 += 2.0 * 16.0 * n * I.n_ig;          // partial sums out and back
    }
    if (flops_out) {
        flops_out[0] = f0;
        flops_out[1] = f1;
        flops_out[2] = f2;
    }
    if (bytes_out) {
        bytes_out[0] = b0;
        bytes_out[1] = b1;
        bytes_out[2] = b2;
    }
    return WKE_OK;
}

}  // extern "C"

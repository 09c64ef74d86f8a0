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
#include "wke_layout.hpp"

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

}  // namespace

// A plan: its host-side layout (wke_layout.hpp) and its device memory.
struct wke_plan_s : PlanLayout {
    hipStream_t stream = nullptr;
    int device = 0;
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
    FieldRef* d_flds = nullptr;
    int* d_uofs = nullptr;
    int* d_sub = nullptr;              // fused form: slab-field subsets of the item groups
    double* d_kt64 = nullptr;          // 2D axis-1 interpolation kernels of the slab fields
    float* d_kt32 = nullptr;
    std::vector<void*> allocs;
    // instances of different N are independent: each N group can run on a
    // stream of its own, forked from and joined back to the plan's stream
    // with events (wke_plan_set_concurrency; on by default when the plan has
    // more than one group)
    bool concurrent = false;
    std::vector<hipStream_t> gstream;
    hipEvent_t ev_fork = nullptr;
    std::vector<hipEvent_t> ev_join;
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
    std::string err;
    const wke_status st = validate_descs(insts, batch, precision, &err);
    return st == WKE_OK ? WKE_OK : fail(st, "%s", err.c_str());
}

wke_status check(const wke_plan_s* p) {
    const std::string err = check_layout(*p);
    if (!err.empty()) return fail(WKE_ERR_INVALID, "internal: plan layout: %s", err.c_str());
    return WKE_OK;
}

wke_status build_plan(wke_plan_s* p, const wke_desc* insts, int batch, int precision) {
    HIP_TRY(hipGetDevice(&p->device));
    layout_instances(p, insts, batch, precision, p->nyq);
    WKE_TRY(check(p));

    // device allocations
    WKE_TRY(dev_alloc(p, &p->d_inst, batch));
    WKE_TRY(dev_alloc(p, &p->d_nodes, p->n_nodes));
    std::vector<UnitPat> allpat;
    for (int i = 0; i < batch; ++i) allpat.insert(allpat.end(), p->pats[i].begin(), p->pats[i].end());
    WKE_TRY(dev_alloc(p, &p->d_upat, allpat.size()));
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
    HIP_TRY(hipMemcpyAsync(p->d_upat, allpat.data(), sizeof(UnitPat) * allpat.size(), hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(p->d_upat_off, p->pat_off.data(), sizeof(int) * batch, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemsetAsync(p->d_counters, 0, sizeof(unsigned int) * std::max(1, p->n_counters), s));
    for (auto& kv : p->tw_off)
        HIP_TRY(launch_twiddles(kv.first, p->d_tw64 + 2 * kv.second, p->d_tw32 + 2 * kv.second, s));
    for (int i = 0; i < batch; ++i)
        HIP_TRY(launch_tables(p->d_inst, p->inst[i], i, p->d_nodes, p->d_upat + p->pat_off[i], p->d_ph64, p->d_ph32,
                              p->d_uw64, p->d_uw32, s));
    // the host copies above read pageable buffers owned by this function
    HIP_TRY(hipStreamSynchronize(s));

    // shared slab fields: read back the quadrature, find the shifts that
    // agree on axes 1..d-1 and the distinct shift vectors, and size the
    // tables they index
    std::vector<double> nodes(std::max<long long>(1, p->n_nodes));
    HIP_TRY(hipMemcpy(nodes.data(), p->d_nodes, sizeof(double) * p->n_nodes, hipMemcpyDeviceToHost));
    layout_fields(p, nodes.data());
    WKE_TRY(check(p));
    if (precision == WKE_F64) {
        double* b;
        WKE_TRY(dev_alloc(p, &b, 2 * p->n_G));
        p->d_G = b;
    } else {
        float* b;
        WKE_TRY(dev_alloc(p, &b, 2 * p->n_G));
        p->d_G = b;
    }
    std::vector<int> allrep, allhid(std::max<long long>(1, p->n_hid), 0);
    for (int i = 0; i < batch; ++i) {
        allrep.insert(allrep.end(), p->hrep[i].begin(), p->hrep[i].end());
        std::copy(p->hid[i].begin(), p->hid[i].end(), allhid.begin() + p->inst[i].off_hid);
    }
    WKE_TRY(dev_alloc(p, &p->d_hrep, allrep.size()));
    WKE_TRY(dev_alloc(p, &p->d_hid, allhid.size()));
    WKE_TRY(dev_alloc(p, &p->d_rounds, std::max<long long>(1, p->n_rounds)));
    WKE_TRY(dev_alloc(p, &p->d_flds, std::max<size_t>(1, allhid.size())));
    WKE_TRY(dev_alloc(p, &p->d_uofs, std::max<size_t>(1, allhid.size())));
    WKE_TRY(dev_alloc(p, &p->d_sub, std::max<long long>(1, p->n_sub)));
    HIP_TRY(hipMemcpyAsync(p->d_hrep, allrep.data(), sizeof(int) * allrep.size(), hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(p->d_hid, allhid.data(), sizeof(int) * allhid.size(), hipMemcpyHostToDevice, s));
    // interpolation kernels of the 2D slab fields (the fused column pass)
    WKE_TRY(dev_alloc(p, &p->d_kt64, 2 * std::max<long long>(1, p->n_kt)));
    if (precision == WKE_F32) WKE_TRY(dev_alloc(p, &p->d_kt32, 2 * std::max<long long>(1, p->n_kt)));
    HIP_TRY(hipMemcpyAsync(p->d_inst, p->inst.data(), sizeof(InstDev) * batch, hipMemcpyHostToDevice, s));
    for (int i = 0; i < batch; ++i)
        HIP_TRY(launch_ktab(p->d_inst, p->inst[i], i, p->d_ph64, p->d_hrep, p->d_kt64, p->d_kt32, s));

    // tasks, grouped by N
    layout_tasks(p);
    for (Group& G : p->groups) {
        if (p->nyq && !G.colkind)
            return fail(WKE_ERR_UNSUPPORTED, "the real form needs the field-parallel column pass (at most %d product "
                        "units per item and one item's fields in a workgroup)", FP_MAX_UNITS);
        WKE_TRY(dev_alloc(p, &G.dA, G.maxA));
        WKE_TRY(dev_alloc(p, &G.dB, G.maxB));
        WKE_TRY(dev_alloc(p, &G.dF, G.hF.size()));
        HIP_TRY(hipMemcpyAsync(G.dA, G.hA.data(), sizeof(TaskA) * G.hA.size(), hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(G.dF, G.hF.data(), sizeof(TaskB) * G.hF.size(), hipMemcpyHostToDevice, s));
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
    for (hipStream_t gs : p->gstream) (void)hipStreamDestroy(gs);
    for (hipEvent_t e : p->ev_join) (void)hipEventDestroy(e);
    if (p->ev_fork) (void)hipEventDestroy(p->ev_fork);
    for (void* q : p->allocs) (void)hipFree(q);
    delete p;
}

// Column-pass tasks and field-parallel rounds for the group's current
// splits, checked and uploaded (waits for the plan's stream first).
wke_status apply_split(wke_plan_s* p, Group& G) {
    layout_split(p, G);
    if (!launch_fits(G))
        return fail(WKE_ERR_UNSUPPORTED, "the column-pass form and work split chosen for N = %d do not fit one "
                    "workgroup (%d lanes, %u bytes of LDS)", G.N, G.fp_threads, G.fp_lds);
    WKE_TRY(check(p));
    HIP_TRY(hipStreamSynchronize(p->stream));
    HIP_TRY(hipMemcpy(p->d_inst, p->inst.data(), sizeof(InstDev) * p->batch, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(G.dB, G.hB.data(), sizeof(TaskB) * G.hB.size(), hipMemcpyHostToDevice));
    for (int i = 0; i < p->batch; ++i) {
        if (p->inst[i].N != G.N || p->rounds[i].empty()) continue;
        const InstDev& I = p->inst[i];
        if (p->rounds_fused[i]) {
            const long long n = (long long)p->max_ig[i] * (1 + I.n_slab);
            HIP_TRY(hipMemcpy(p->d_sub + p->sub_off[i], p->sub.data() + p->sub_off[i], sizeof(int) * n,
                              hipMemcpyHostToDevice));
        }
        HIP_TRY(hipMemcpy(p->d_rounds + I.off_rounds, p->rounds[i].data(), sizeof(RoundDesc) * p->rounds[i].size(),
                          hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(p->d_flds + I.off_hid, p->flds[i].data(), sizeof(FieldRef) * p->flds[i].size(),
                          hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(p->d_uofs + I.off_hid, p->uofs[i].data(), sizeof(int) * p->uofs[i].size(),
                          hipMemcpyHostToDevice));
    }
    return WKE_OK;
}

const void* ph_ptr(const wke_plan_s* p) { return p->prec == WKE_F64 ? (const void*)p->d_ph64 : (const void*)p->d_ph32; }
const void* uw_ptr(const wke_plan_s* p) { return p->prec == WKE_F64 ? (const void*)p->d_uw64 : (const void*)p->d_uw32; }
const void* tw_ptr(const wke_plan_s* p) { return p->prec == WKE_F64 ? (const void*)p->d_tw64 : (const void*)p->d_tw32; }

hipError_t group_colfwd(wke_plan_s* p, Group& G, const double* f, hipStream_t s) {
    // the fused column pass reads spec0 column-major
    ColFwdArgs a{p->d_inst, G.dF, f, p->d_spec0, tw_ptr(p), G.colkind == 2 ? 1 : 0};
    return launch_colfwd(p->prec, p->d, G.N, a, (int)G.hF.size(), s);
}

wke_status run_colfwd(wke_plan_s* p, const double* f) {
    for (Group& G : p->groups) HIP_TRY(group_colfwd(p, G, f, p->stream));
    return WKE_OK;
}

hipError_t group_passA(wke_plan_s* p, Group& G, const LaunchEvents* ev = nullptr, hipStream_t s = nullptr) {
    if (G.colkind == 2) return hipSuccess;       // the fused column pass builds its slab fields itself
    PassAArgs a{p->d_inst, G.dA, p->d_spec0, p->d_G, ph_ptr(p), p->d_hrep, tw_ptr(p), G.slab_alt};
    return launch_passA(p->prec, p->d, G.N, a, (int)G.hA.size(), ev || !s ? p->stream : s, ev);
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
    a.uofs = p->d_uofs;
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
    a.fp_mfma = G.colkind == 2 ? G.fp_mfma : 0;
    a.one = p->batch == 1 && p->inst[0].n_ig == 1 && !G.hB.empty() ? 1 : 0;
    if (a.one) a.task1 = G.hB[0];
    a.fp_off_h = G.fp_off_h;
    a.fp_off_ph = G.fp_off_ph;
    a.kt = p->prec == WKE_F64 ? (const void*)p->d_kt64 : (const void*)p->d_kt32;
    a.sub = p->d_sub;
    a.real = p->nyq;
    return a;
}

hipError_t group_passB(wke_plan_s* p, Group& G, int mode, int stage, const double* F0, double* out, double* y,
                       double dt, hipStream_t s) {
    const PassBArgs a = passB_args(p, G, mode, stage, F0, out, y, dt);
    return launch_passB(p->prec, p->d, G.N, a, (int)G.hB.size(), s);
}

// Enqueue fn(G, stream) for every N group.  Concurrent plans run each group
// on its own stream: the group streams wait for an event recorded on the
// plan's stream, and the plan's stream waits for an event recorded on each
// group stream after its work, so that the call stays ordered with the
// caller's work on the plan's stream (and, under graph capture, the groups
// become parallel branches of the captured graph).
template <class Fn> wke_status for_groups(wke_plan_s* p, Fn fn) {
    const size_t ng = p->groups.size();
    if (!p->concurrent || ng < 2) {
        for (Group& G : p->groups) WKE_TRY(fn(G, p->stream));
        return WKE_OK;
    }
    if (p->gstream.size() != ng) {
        // created on first use, at the default priority
        while (p->gstream.size() < ng) {
            hipStream_t gs = nullptr;
            HIP_TRY(hipStreamCreateWithFlags(&gs, hipStreamNonBlocking));
            p->gstream.push_back(gs);
            hipEvent_t e = nullptr;
            HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
            p->ev_join.push_back(e);
        }
        if (!p->ev_fork) HIP_TRY(hipEventCreateWithFlags(&p->ev_fork, hipEventDisableTiming));
    }
    HIP_TRY(hipEventRecord(p->ev_fork, p->stream));
    for (size_t g = 0; g < ng; ++g) {
        HIP_TRY(hipStreamWaitEvent(p->gstream[g], p->ev_fork, 0));
        WKE_TRY(fn(p->groups[g], p->gstream[g]));
        HIP_TRY(hipEventRecord(p->ev_join[g], p->gstream[g]));
    }
    for (size_t g = 0; g < ng; ++g) HIP_TRY(hipStreamWaitEvent(p->stream, p->ev_join[g], 0));
    return WKE_OK;
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
    p->concurrent = p->groups.size() > 1;
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
    p->concurrent = p->groups.size() > 1;
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
    return for_groups(p, [&](Group& G, hipStream_t s) -> wke_status {
        HIP_TRY(group_colfwd(p, G, f, s));
        HIP_TRY(group_passA(p, G, nullptr, s));
        HIP_TRY(group_passB(p, G, MODE_EVAL, 0, f, Q, nullptr, 0.0, s));
        return WKE_OK;
    });
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

// The RK4 stages of one group (slab and column pass per stage) on stream s.
wke_status group_rk_steps(wke_plan_s* p, Group& G, double* f, double dt, int nsteps, hipStream_t s) {
    for (int n = 0; n < nsteps; ++n)
        for (int st = 0; st < 4; ++st) {
            HIP_TRY(group_passA(p, G, nullptr, s));
            HIP_TRY(group_passB(p, G, MODE_RK, st, st == 0 ? f : p->d_ystage, nullptr, f, dt, s));
        }
    return WKE_OK;
}

wke_status enqueue_rk_step(wke_plan_s* p, double* f, double dt) {
    return for_groups(p, [&](Group& G, hipStream_t s) { return group_rk_steps(p, G, f, dt, 1, s); });
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
    if (p->use_graphs) {
        WKE_TRY(for_groups(p, [&](Group& G, hipStream_t s) -> wke_status {
            HIP_TRY(group_colfwd(p, G, f, s));
            return WKE_OK;
        }));
        if (!p->step_exec || p->graph_f != f || p->graph_dt != dt) WKE_TRY(capture_step(p, f, dt));
        for (int n = 0; n < nsteps; ++n) HIP_TRY(hipGraphLaunch(p->step_exec, p->stream));
        return WKE_OK;
    }
    // each group runs all its steps on its stream before joining
    return for_groups(p, [&](Group& G, hipStream_t s) -> wke_status {
        HIP_TRY(group_colfwd(p, G, f, s));
        return group_rk_steps(p, G, f, dt, nsteps, s);
    });
}

wke_status wke_plan_set_concurrency(wke_plan_t p, int enable) {
    if (!p) return fail(WKE_ERR_INVALID, "NULL plan");
    if (p->concurrent != (enable != 0)) drop_graph(p);     // the captured step follows the mode
    p->concurrent = enable != 0;
    return WKE_OK;
}

int wke_plan_groups(wke_plan_t p) { return p ? (int)p->groups.size() : 0; }

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
        // also the first few splits whose column-pass tasks fill whole waves
        // of one workgroup per compute unit (the plans with many items run
        // one large workgroup per compute unit at a time, and a last,
        // partial wave of workgroups leaves compute units idle)
        long long ncb = 0;
        int lo = cap;
        for (int i = 0; i < p->batch; ++i)
            if (p->inst[i].N == G.N) {
                ncb += p->inst[i].n_cb;
                lo = std::min(lo, p->min_ig[i]);
            }
        for (int n = std::max(1, lo), added = 0; n <= cap && added < 3; ++n)
            if ((ncb * n) % 256 == 0 && std::find(splits.begin(), splits.end(), n) == splits.end()) {
                splits.push_back(n);
                ++added;
            }
        // 0 item slots; 1, 2 field-parallel narrow, wide; 3, 4 fused narrow,
        // wide; 5, 6 field-parallel narrow, wide in half-width rounds; 7, 8
        // fused on the matrix cores, narrow, wide.
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
            if (fused_width_ok(p, G, 0, 1)) kinds.push_back(7);
            if (fused_width_ok(p, G, 1, 1)) kinds.push_back(8);
            if (fp_feasible(p, G, 1)) {
                kinds.push_back(5);
                kinds.push_back(6);
            }
        }
        double best_us = 1e300;
        int best = splits[0], best_kind = kinds.empty() ? 0 : kinds[0];
        auto set_kind = [&](int kind) {
            G.colkind = kind == 0 ? 0 : (kind == 3 || kind == 4 || kind >= 7 ? 2 : 1);
            G.fp_wide = kind == 2 || kind == 4 || kind == 6 || kind == 8 ? 1 : 0;
            G.fp_half = kind == 5 || kind == 6 ? 1 : 0;
            G.fp_mfma = kind >= 7 ? 1 : 0;
        };
        std::map<int, int> ng_full;     // split -> most fields in a round at full width
        for (int kind : kinds) {
            for (int n : splits) {
                for (int i = 0; i < p->batch; ++i)
                    if (p->inst[i].N == G.N) set_split(p, i, n);
                // half rounds that would hold the same fields as full ones
                // are the same launch: not timed again
                if ((kind == 5 || kind == 6) && ng_full.count(n) && ng_full[n] <= fp_field_cap(p, G.N, 1)) continue;
                set_kind(kind);
                st = apply_split(p, G);
                if (st == WKE_ERR_UNSUPPORTED) {       // this form does not fit at this split
                    st = WKE_OK;
                    continue;
                }
                if (st != WKE_OK) break;
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
        set_kind(best_kind);
        if ((st = apply_split(p, G)) != WKE_OK) break;
        // the 3D slab pass's workgroup width (fields transformed at once),
        // where two are built, timed alone and the faster kept
        if (G.colkind != 2 && slab_alt_available(p, G)) {
            double alt_us[2] = {0.0, 0.0};
            for (int alt = 0; alt < 2 && st == WKE_OK; ++alt) {
                layout_slab_tasks(p, G, alt);
                hipError_t e = hipMemcpyAsync(G.dA, G.hA.data(), sizeof(TaskA) * G.hA.size(), hipMemcpyHostToDevice,
                                              p->stream);
                if (e == hipSuccess) e = group_passA(p, G);                                   // warm
                if (e == hipSuccess) e = hipEventRecord(e0, p->stream);
                for (int r = 0; r < reps && e == hipSuccess; ++r) e = group_passA(p, G);
                if (e == hipSuccess) e = hipEventRecord(e1, p->stream);
                if (e == hipSuccess) e = hipEventSynchronize(e1);
                float ms = 0.f;
                if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
                if (e != hipSuccess) st = fail(WKE_ERR_HIP, "tuning launch failed: %s", hipGetErrorString(e));
                alt_us[alt] = 1000.0 * ms / reps;
            }
            if (st != WKE_OK) break;
            layout_slab_tasks(p, G, alt_us[1] < alt_us[0] ? 1 : 0);
            HIP_TRY(hipMemcpyAsync(G.dA, G.hA.data(), sizeof(TaskA) * G.hA.size(), hipMemcpyHostToDevice, p->stream));
            WKE_TRY(check(p));
        }
        if (us_out) {
            us_out[3 * gi] = G.colkind == 1 && G.fp_half ? WKE_COLUMN_FIELDS_HALF
                             : G.colkind == 2 && G.fp_mfma ? WKE_COLUMN_FUSED_MFMA : G.colkind;
            us_out[3 * gi + 1] = best;
            us_out[3 * gi + 2] = best_us;
        }
        ++gi;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return st;
}

}  // extern "C"

namespace {

// The column-pass choices of a plan, to restore when a new one is refused.
struct ColumnState {
    std::vector<InstDev> inst;
    std::vector<Group> groups;
};

ColumnState save_columns(const wke_plan_s* p) { return ColumnState{p->inst, p->groups}; }

// Put the saved choices back (and their tasks and rounds on the device),
// then return the status of the refusal.
wke_status restore_columns(wke_plan_s* p, const ColumnState& c, wke_status refusal) {
    const std::string msg = g_last_error;
    p->inst = c.inst;
    for (size_t g = 0; g < p->groups.size(); ++g) {
        Group& G = p->groups[g];
        G.colkind = c.groups[g].colkind;
        G.fp_wide = c.groups[g].fp_wide;
        G.fp_half = c.groups[g].fp_half;
        G.fp_mfma = c.groups[g].fp_mfma;
        WKE_TRY(apply_split(p, G));
    }
    g_last_error = msg;
    return refusal;
}

}  // namespace

extern "C" {

wke_status wke_plan_set_split(wke_plan_t p, int n) {
    if (!p || n < 1) return fail(WKE_ERR_INVALID, "bad arguments");
    if (p->fine) return wke_plan_set_split(p->fine, n);
    drop_graph(p);
    const ColumnState saved = save_columns(p);
    for (Group& G : p->groups) {
        for (int i = 0; i < p->batch; ++i)
            if (p->inst[i].N == G.N) set_split(p, i, n);
        const wke_status st = apply_split(p, G);
        if (st == WKE_ERR_UNSUPPORTED) return restore_columns(p, saved, st);
        WKE_TRY(st);
    }
    return WKE_OK;
}

wke_status wke_plan_set_column_kernel(wke_plan_t p, int kind) {
    if (!p || (kind != WKE_COLUMN_SLOTS && kind != WKE_COLUMN_FIELDS && kind != WKE_COLUMN_FUSED &&
               kind != WKE_COLUMN_FIELDS_HALF && kind != WKE_COLUMN_FUSED_MFMA))
        return fail(WKE_ERR_INVALID, "bad arguments");
    const int mfma = kind == WKE_COLUMN_FUSED_MFMA ? 1 : 0;
    if (mfma) kind = WKE_COLUMN_FUSED;
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
            if (!fused_feasible(p, G, mfma))
                return fail(WKE_ERR_UNSUPPORTED, "the fused column pass needs d = 2, the field-parallel form "
                            "and at most %d slab fields", FUSED_MAX_SLAB);
    drop_graph(p);
    HIP_TRY(hipStreamSynchronize(p->stream));
    const ColumnState saved = save_columns(p);
    for (Group& G : p->groups) {
        if (kind == WKE_COLUMN_FUSED) G.fp_wide = fused_width_ok(p, G, 1, mfma) ? 1 : 0;
        G.fp_mfma = mfma;
        G.fp_half = kind == WKE_COLUMN_FIELDS_HALF ? 1 : 0;
        G.colkind = kind == WKE_COLUMN_FIELDS_HALF ? WKE_COLUMN_FIELDS : kind;
        const wke_status st = apply_split(p, G);
        if (st == WKE_ERR_UNSUPPORTED) return restore_columns(p, saved, st);
        WKE_TRY(st);
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

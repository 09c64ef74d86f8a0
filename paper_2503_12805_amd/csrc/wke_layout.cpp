// Host-side plan layout (see wke_layout.hpp).  Plain C++17.
#include "wke_layout.hpp"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>

#include "wke_shape.hpp"

namespace wke {

// ---------------------------------------------------------------------------
// Launch geometry of the template instances.
// ---------------------------------------------------------------------------
namespace {

int tpt_of(int N) {
    switch (N) {
        case 16: return FftShape<16>::TPT;
        case 32: return FftShape<32>::TPT;
        case 48: return FftShape<48>::TPT;
        case 64: return FftShape<64>::TPT;
        case 96: return FftShape<96>::TPT;
        case 128: return FftShape<128>::TPT;
    }
    return 0;
}

// LDS slots of one column transform's scratch in the field-parallel column
// pass (col_slots)
int slots_of(int d, int N) {
    switch (N) {
        case 16: return d == 3 ? col_slots<3, 16>() : col_slots<2, 16>();
        case 32: return d == 3 ? col_slots<3, 32>() : col_slots<2, 32>();
        case 48: return d == 3 ? col_slots<3, 48>() : col_slots<2, 48>();
        case 64: return d == 3 ? col_slots<3, 64>() : col_slots<2, 64>();
        case 96: return d == 3 ? col_slots<3, 96>() : col_slots<2, 96>();
        case 128: return d == 3 ? col_slots<3, 128>() : col_slots<2, 128>();
    }
    return 0;
}

// LDS offset, from a point's own slot, of round-local field k in the
// column pass's field blocks (fp_block(d) columns of slots_of(d, N) slots
// each): block k in complex slots, or in the real form, where two fields
// share a block as its real and imaginary parts, block k / 2 counted in
// real components
int factor_offset(int d, int N, bool real, int k) {
    const int bs = fp_block(d) * slots_of(d, N);
    return real ? 2 * (k >> 1) * bs + (k & 1) : k * bs;
}

}  // namespace

int fp_columns(int d) { return fp_block(d); }

unsigned fp_lds_bytes(int prec, int d, int N, int nt, int ng) {
    const int tpt = tpt_of(N), gb = fp_block(d);
    if (tpt == 0 || nt <= 0) return 0;
    const size_t sz = prec == 0 ? 16 : 8;
    const size_t slots = (size_t)slots_of(d, N);       // transform scratch per column
    const size_t pts = (size_t)gb * N;                 // grid points of a workgroup
    const size_t fields = (size_t)ng * gb * slots * sz;
    const size_t tail = (size_t)(nt / pts) * pts * 16 + (pts + gb * slots) * sz;
    return (unsigned)(fields > tail ? fields : tail);
}

int fp_group_cap(int prec, int d, int N, bool fused, bool real) {
    const int tpt = tpt_of(N), gb = fp_block(d);
    if (tpt == 0) return 0;
    const int by_lanes = fp_max_threads(prec, N, fused, real) / (gb * tpt);
    const int by_lds = (int)(FP_LDS_LIMIT / ((prec == 0 ? 16 : 8) * gb * slots_of(d, N)));
    return by_lanes < by_lds ? by_lanes : by_lds;
}

int fused_chunks(int prec, int N, int nt) {
    // chunks of the sum over x1, as many as the workgroup has lanes for (up
    // to 8), each a multiple of 8 terms; 0 if none fits
    (void)prec;
    int best = 0;
    for (int w = 1; w <= 8; ++w)
        if (N % w == 0 && (N / w) % 8 == 0 && w * N <= nt) best = w;
    return best;
}

unsigned fused_lds_bytes(int prec, int N, int nt, int ng, int ns, int nparts, unsigned* off_h) {
    const size_t sz = prec == 0 ? 16 : 8;
    size_t a = fp_lds_bytes(prec, 2, N, nt, ng);
    const size_t p1 = (size_t)nparts * ns * fused_ppitch(prec, N) * sz;
    if (p1 > a) a = p1;
    a = (a + 15) / 16 * 16;
    if (off_h) *off_h = (unsigned)a;
    // the slab-field columns (padded rows), then the gathered kernels
    return (unsigned)(a + (size_t)ns * (fused_hpitch(N) + N) * sz);
}

int fp_threads(int prec, int d, int N, int ng, int kp, bool fused, bool real) {
    const int tpt = tpt_of(N), gb = fp_block(d);
    if (tpt == 0 || ng <= 0) return 0;
    const int cap = fp_max_threads(prec, N, fused, real);
    for (; kp >= 1; --kp) {
        int nt = ng * gb * tpt > gb * N * kp ? ng * gb * tpt : gb * N * kp;
        nt = ((nt + 63) / 64) * 64;
        if (nt <= cap && fp_lds_bytes(prec, d, N, nt, ng) <= FP_LDS_LIMIT) return nt;
    }
    return 0;
}

bool geometry_of(int prec, int d, int N, Geometry* g) {
#define WKE_GEO(DD, NN)                                                        \
    if (d == DD && N == NN) {                                                  \
        g->tpt = Geo<DD, NN>::TPT;                                             \
        g->groups_b = Geo<DD, NN>::GB;                                         \
        g->slots_b = prec == 0 ? Geo<DD, NN>::IGS64 : Geo<DD, NN>::IGS32;      \
        g->groups_f = Geo<DD, NN>::GF;                                         \
        g->groups_a = DD == 2 ? (prec == 0 ? Geo<DD, NN>::JB64 : Geo<DD, NN>::JB32) : 1;   \
        g->shifts_per_task_a = DD == 2 ? (prec == 0 ? Geo<DD, NN>::SB64 : Geo<DD, NN>::SB32) \
                                       : (prec == 0 ? Geo<DD, NN>::SPT3_64 : Geo<DD, NN>::SPT3_32); \
        g->shifts_per_task_a_alt = prec == 0 && !Geo<DD, NN>::REG3_64 ? Geo<DD, NN>::SC64_ALT : 0; \
        return true;                                                           \
    }
    WKE_GEO(2, 16) WKE_GEO(2, 32) WKE_GEO(2, 48) WKE_GEO(2, 64) WKE_GEO(2, 96) WKE_GEO(2, 128)
    WKE_GEO(3, 16) WKE_GEO(3, 32) WKE_GEO(3, 64)
#undef WKE_GEO
    return false;
}

// ---------------------------------------------------------------------------
// Descriptors.
// ---------------------------------------------------------------------------
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

namespace {

wke_status bad(std::string* err, wke_status s, const char* fmt, int i, int v = 0, int w = 0) {
    char buf[256];
    std::snprintf(buf, sizeof buf, fmt, i, v, w);
    if (err) *err = buf;
    return s;
}

}  // namespace

wke_status validate_descs(const wke_desc* insts, int batch, int precision, std::string* err) {
    if (!insts || batch < 1) return bad(err, WKE_ERR_INVALID, "need at least one instance", 0);
    if (precision != WKE_F64 && precision != WKE_F32)
        return bad(err, WKE_ERR_INVALID, "precision must be WKE_F64 or WKE_F32", 0);
    const int d0 = insts[0].d;
    for (int i = 0; i < batch; ++i) {
        const wke_desc& q = insts[i];
        if (q.d != 2 && q.d != 3) return bad(err, WKE_ERR_INVALID, "instance %d: d must be 2 or 3", i);
        if (q.d != d0) return bad(err, WKE_ERR_INVALID, "instance %d: all instances of a plan must share d", i);
        if (q.N < 2 || (q.N & 1)) return bad(err, WKE_ERR_INVALID, "instance %d: N must be even and >= 2", i);
        if (!supported_N(q.d, q.N))
            return bad(err, WKE_ERR_UNSUPPORTED, "instance %d: N = %d is not built for d = %d", i, q.N, q.d);
        if (!(q.L > 0.0) || !std::isfinite(q.L)) return bad(err, WKE_ERR_INVALID, "instance %d: L must be positive", i);
        if (!std::isfinite(q.R)) return bad(err, WKE_ERR_INVALID, "instance %d: R must be finite", i);
        if (q.N_r < 1 || q.N_s < 1 || q.N_sig < 1)
            return bad(err, WKE_ERR_INVALID, "instance %d: quadrature counts must be >= 1", i);
        if (q.N_r > 4096) return bad(err, WKE_ERR_INVALID, "instance %d: N_r too large", i);
        if (q.d == 2) {
            if (q.sphere_rule != WKE_MIDPOINT) return bad(err, WKE_ERR_INVALID, "instance %d: 2D uses WKE_MIDPOINT", i);
            if (q.N_s > 4096 || q.N_sig > 4096) return bad(err, WKE_ERR_INVALID, "instance %d: angle counts too large", i);
        } else {
            const int np = rule_points(q.sphere_rule);
            if (!np) return bad(err, WKE_ERR_INVALID, "instance %d: 3D needs a spherical design rule", i);
            if (q.N_s != np || q.N_sig != np)
                return bad(err, WKE_ERR_INVALID, "instance %d: N_s and N_sig must equal the design's %d points", i, np);
        }
        const double R = q.R > 0 ? q.R : 4.0 * q.L / (3.0 + std::sqrt(2.0));
        if (R > 2.0 * q.L) return bad(err, WKE_ERR_INVALID, "instance %d: R must not exceed 2L", i);
    }
    return WKE_OK;
}

// ---------------------------------------------------------------------------
// Shared fields.
// ---------------------------------------------------------------------------
namespace {

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

long long columns_of(const InstDev& I) { return I.d == 2 ? I.N : (long long)I.N * I.N; }

}  // namespace

// ---------------------------------------------------------------------------
// Layout steps.
// ---------------------------------------------------------------------------
void layout_instances(PlanLayout* L, const wke_desc* insts, int batch, int precision, int nyq) {
    L->batch = batch;
    L->prec = precision;
    L->d = insts[0].d;
    L->nyq = nyq;
    L->desc.assign(insts, insts + batch);

    // distinct N values, in order of first appearance
    std::vector<int> Ns;
    for (int i = 0; i < batch; ++i)
        if (std::find(Ns.begin(), Ns.end(), insts[i].N) == Ns.end()) Ns.push_back(insts[i].N);
    for (int N : Ns) {
        L->tw_off[N] = L->n_tw;
        L->n_tw += N;
    }

    int total_pass_b_cb = 0;
    for (int i = 0; i < batch; ++i) {
        Geometry g;
        geometry_of(precision, insts[i].d, insts[i].N, &g);
        const long long C = insts[i].d == 2 ? insts[i].N : (long long)insts[i].N * insts[i].N;
        total_pass_b_cb += (int)((C + g.groups_b - 1) / g.groups_b);
    }

    L->inst.resize(batch);
    L->pats.resize(batch);
    L->pat_off.assign(batch, 0);
    L->max_ig.assign(batch, 1);
    L->min_ig.assign(batch, 1);
    long long off_state = 0;
    int counter_off = 0, npat = 0;
    for (int i = 0; i < batch; ++i) {
        const wke_desc& q = insts[i];
        InstDev& I = L->inst[i];
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
        std::vector<UnitPat>& pat = L->pats[i];
        pat.clear();
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
        L->pat_off[i] = npat;
        npat += (int)pat.size();
        I.U_item = (int)pat.size();
        I.n_items = q.N_r * q.N_s;
        I.n_shift = I.n_items * I.S_item;
        I.n_unit = I.n_items * I.U_item;
        const long long C = columns_of(I);
        I.n_cb = (int)((C + g.groups_b - 1) / g.groups_b);
        // split the quadrature sum over enough workgroups to fill the chip,
        // but give every item slot of a workgroup at least one item; the
        // field-parallel 2D form may split further (up to 8 groups)
        const int slot_ig = std::max(1, (I.n_items + g.slots_b - 1) / g.slots_b);
        // a workgroup stages its items' slab-field indices in LDS (HID_CAP)
        // (the real form adds the zero shift to every round's fields)
        const int s_cap = HID_CAP / (I.S_item + nyq);
        const int min_ig = (I.n_items + s_cap - 1) / s_cap;
        const int max_ig = std::max(min_ig, q.d == 2 ? std::max(slot_ig, std::min(I.n_items, 8)) : slot_ig);
        L->max_ig[i] = max_ig;
        L->min_ig[i] = min_ig;
        const int want = std::max(1, (256 + total_pass_b_cb - 1) / total_pass_b_cb);
        I.n_ig = std::max(min_ig, std::min(slot_ig, want));
        I.items_per_ig = (I.n_items + I.n_ig - 1) / I.n_ig;
        I.n_ig = (I.n_items + I.items_per_ig - 1) / I.items_per_ig;
        I.counter_off = counter_off;
        counter_off += (int)C;          // room for one arrival counter per column
        I.off_state = off_state;
        I.off_spec0 = off_state;
        off_state += np;
        I.off_nodes = L->n_nodes;
        L->n_nodes += 2LL * q.N_r + (long long)(q.d + 1) * (q.N_s + q.N_sig);
        I.nyq_zero = nyq;
        I.off_ph = L->n_ph;
        L->n_ph += (long long)(I.n_shift + nyq) * q.d * q.N;
        I.off_unit = L->n_unit;
        L->n_unit += I.n_unit;
        I.off_part = L->n_part;
        if (max_ig > 1) L->n_part += (long long)max_ig * np;   // room for any split
        I.off_tw = L->tw_off[q.N];
    }
    L->total_elems = (size_t)off_state;
    L->n_spec0 = off_state;
    L->n_counters = counter_off;

    L->groups.clear();
    for (int N : Ns) {
        Group G;
        G.N = N;
        L->groups.push_back(std::move(G));
    }
}

void layout_fields(PlanLayout* L, const double* nodes) {
    const int batch = L->batch;
    L->hrep.resize(batch);
    L->hid.resize(batch);
    L->frep.resize(batch);
    L->fid.resize(batch);
    L->rounds.resize(batch);
    L->flds.resize(batch);
    L->lidx.resize(batch);
    L->uofs.resize(batch);
    L->ig_r0.resize(batch);
    L->ig_r1.resize(batch);
    L->ig_f0.resize(batch);
    L->ig_nfl.resize(batch);
    L->fp_ng.assign(batch, 0);
    L->fp_ni.assign(batch, 0);
    L->n_G = L->n_hrep = L->n_hid = L->n_rounds = L->n_kt = 0;
    for (int i = 0; i < batch; ++i) {
        InstDev& I = L->inst[i];
        group_shifts(I, nodes + I.off_nodes, 1, &L->hrep[i], &L->hid[i]);
        group_shifts(I, nodes + I.off_nodes, 0, &L->frep[i], &L->fid[i]);
        // the slab-field count first: the sizes below depend on it
        I.n_slab = (int)L->hrep[i].size();
        I.off_rounds = L->n_rounds;
        L->n_rounds += I.n_items;
        I.off_kt = L->n_kt;
        if (I.d == 2) L->n_kt += 2LL * I.n_slab * I.N;      // each row twice over
        I.off_G = L->n_G;
        L->n_G += (long long)I.n_slab * I.n_pts;
        I.off_hrep = L->n_hrep;
        L->n_hrep += I.n_slab;
        I.off_hid = L->n_hid;
        // per shift (and the zero shift); the real form's rounds hold up to
        // one more field each, and there are at most n_items rounds
        L->n_hid += I.n_shift + (long long)I.nyq_zero * (1 + I.n_items);
    }
    // the fused form's slab-field subsets: room for every split
    L->sub_off.assign(batch, 0);
    L->ig_sub.assign(batch, {});
    L->rounds_fused.assign(batch, 0);
    L->fp_ns.assign(batch, 0);
    L->n_sub = 0;
    for (int i = 0; i < batch; ++i) {
        L->sub_off[i] = L->n_sub;
        L->n_sub += (long long)L->max_ig[i] * (1 + L->inst[i].n_slab);
        L->fp_ns[i] = L->inst[i].n_slab;
    }
    L->sub.assign(std::max<long long>(1, L->n_sub), 0);
}

// Slab-pass tasks of group G.  alt < 0: the alternative 3D workgroup width
// where it is the wider one and brings a single-instance pass within one
// workgroup per compute unit (the plan's starting choice); alt = 0 or 1:
// the default or the alternative width (the autotuner's).  The alternative
// exists only for some shapes (Geometry::shifts_per_task_a_alt: wider for
// double N = 32); elsewhere alt = 1 acts as 0.
void layout_slab_tasks(PlanLayout* L, Group& G, int alt) {
    const int batch = L->batch;
    G.hA.clear();
    G.slab_alt = 0;
    // 3D: a slab-pass task repeats its slab's forward transform, so it
    // takes as many slab fields as still leaves about SLAB_TASKS tasks for
    // the group (a multiple of the fields a workgroup has in flight)
    constexpr long long SLAB_TASKS = 1024;
    long long slabs = 0;
    for (int i = 0; i < batch; ++i)
        if (L->inst[i].N == G.N) slabs += L->nyq ? G.N / 2 + 1 : G.N;
    const long long per_slab = std::max<long long>(1, SLAB_TASKS / std::max<long long>(1, slabs));
    for (int i = 0; i < batch; ++i) {
        if (L->inst[i].N != G.N) continue;
        const InstDev& I = L->inst[i];
        Geometry g;
        geometry_of(L->prec, I.d, G.N, &g);
        // the real form needs the rows j0 = 0..N/2 only (the others are
        // their conjugates, read mirrored by the column pass)
        const int jend = L->nyq ? G.N / 2 + 1 : G.N;
        // starting choice: the wider alternative where it brings the pass
        // within one workgroup per compute unit (measured at 3D N=32 double
        // with 17 slab fields: 288 -> 192 workgroups, +5% per evaluation;
        // with many slab fields the narrower one is faster)
        const int rows = (jend + g.groups_a - 1) / g.groups_a;
        const int spt0 = g.shifts_per_task_a, spt1 = g.shifts_per_task_a_alt;
        const bool use_alt = spt1 > 0 && (alt < 0 ? spt1 > spt0 && batch == 1 &&
                                                        rows * ((I.n_slab + spt0 - 1) / spt0) > 256 &&
                                                        rows * ((I.n_slab + spt1 - 1) / spt1) <= 256
                                                  : alt > 0);
        if (use_alt) G.slab_alt = 1;
        int spt = use_alt ? spt1 : spt0;
        if (I.d == 3) {
            const long long ntask = std::min<long long>((I.n_slab + spt - 1) / spt, per_slab);
            const int want = (int)((I.n_slab + ntask - 1) / ntask);
            spt = (want + spt - 1) / spt * spt;
        }
        for (int j0 = 0; j0 < jend; j0 += g.groups_a)
            for (int s0 = 0; s0 < I.n_slab; s0 += spt)
                G.hA.push_back(TaskA{i, j0, s0, std::min(I.n_slab, s0 + spt)});
    }
}

bool slab_alt_available(const PlanLayout* L, const Group& G) {
    Geometry g;
    return geometry_of(L->prec, L->d, G.N, &g) && g.shifts_per_task_a_alt > 0;
}

void layout_tasks(PlanLayout* L) {
    const int batch = L->batch;
    for (Group& G : L->groups) {
        G.hF.clear();
        // the device list holds either workgroup width's tasks
        layout_slab_tasks(L, G, 0);
        size_t maxA = G.hA.size();
        if (slab_alt_available(L, G)) {
            layout_slab_tasks(L, G, 1);
            maxA = std::max(maxA, G.hA.size());
        }
        layout_slab_tasks(L, G, -1);
        G.maxA = std::max<size_t>(1, std::max(maxA, G.hA.size()));
        for (int i = 0; i < batch; ++i) {
            if (L->inst[i].N != G.N) continue;
            const InstDev& I = L->inst[i];
            Geometry g;
            geometry_of(L->prec, I.d, G.N, &g);
            const long long C = columns_of(I);
            for (int cb = 0; cb < (int)((C + g.groups_f - 1) / g.groups_f); ++cb)
                G.hF.push_back(TaskB{i, cb, 0, 0, 0, 0, 0, 0});
        }
        size_t maxB = 0;
        for (int i = 0; i < batch; ++i)
            if (L->inst[i].N == G.N) {
                const InstDev& I = L->inst[i];
                const long long C = columns_of(I);
                const int gmin = std::min(fp_columns(I.d), g_slots_columns(L->prec, I.d, I.N));
                maxB += (size_t)((C + gmin - 1) / gmin) * L->max_ig[i];
            }
        G.maxB = std::max<size_t>(1, maxB);
        G.colkind = fp_feasible(L, G) ? 1 : 0;
        size_t nwg = 0;
        for (int i = 0; i < batch; ++i)
            if (L->inst[i].N == G.N) nwg += (size_t)L->inst[i].n_cb * L->inst[i].n_ig;
        G.fp_wide = nwg < 256 ? 1 : 0;
    }
}

// ---------------------------------------------------------------------------
// Column-pass forms and work splits.
// ---------------------------------------------------------------------------

// Distinct fields a field-parallel workgroup holds at once: one per lane
// block, two in the real form (real and imaginary part of one column).
int fp_field_cap(const PlanLayout* L, int N, int half, bool fused) {
    const int g = fp_group_cap(L->prec, L->d, N, fused, L->nyq != 0);
    return (half ? g / 2 : g) * (L->nyq ? 2 : 1);
}

// The field-parallel column pass needs few enough product units per item and
// room for one item's fields in a workgroup.
bool fp_feasible(const PlanLayout* L, const Group& G, int half, bool fused) {
    const int cap = fp_field_cap(L, G.N, half, fused);
    for (const InstDev& I : L->inst) {
        if (I.N != G.N) continue;
        // every round of the real form also holds the zero shift
        if (I.U_item > FP_MAX_UNITS || I.S_item + I.nyq_zero > cap || I.n_items * I.U_item <= 0) return false;
    }
    return cap > 0;
}

// Launch shape of the field-parallel column pass for the group's current
// work split: enough lane groups for one item group's fields (in rounds of
// whole items when they do not fit).
void update_fp(PlanLayout* L, Group& G) {
    G.fp_threads = 0;
    G.fp_lds = 0;
    G.fp_off_h = 0;
    G.fp_off_ph = 0;
    G.fp_nwp = 0;
    if (G.colkind == 0) return;
    int ng = 0, ni = 0;
    for (int i = 0; i < L->batch; ++i)
        if (L->inst[i].N == G.N) {
            ng = std::max(ng, L->fp_ng[i]);
            ni = std::max(ni, L->fp_ni[i]);
        }
    // wide: enough product lanes per point for one item each (up to 16),
    // for few, latency-bound workgroups; narrow: as few lanes as the
    // transforms need, for batches with many workgroups per compute unit
    if (L->nyq) ng = (ng + 1) / 2;         // lane blocks: two fields each in the real form
    G.fp_threads = fp_threads(L->prec, L->d, G.N, ng, G.fp_wide ? std::min(16, std::max(1, ni)) : 1, G.colkind == 2,
                              L->nyq != 0);
    G.fp_lds = fp_lds_bytes(L->prec, L->d, G.N, G.fp_threads, ng);
    if (G.colkind == 2) {
        int ns = 0;
        for (int i = 0; i < L->batch; ++i)
            if (L->inst[i].N == G.N) ns = std::max(ns, L->fp_ns[i]);
        G.fp_nwp = G.fp_mfma ? (G.fp_threads > 0 ? mfma_ksplit(G.N, ns, G.fp_threads) : 0)
                             : fused_chunks(L->prec, G.N, G.fp_threads);
        G.fp_lds = fused_lds_bytes(L->prec, G.N, G.fp_threads, ng, ns, G.fp_nwp, &G.fp_off_h);
        // the first round's phase rows, one (real form: two) per lane block
        const unsigned stage = (unsigned)(ng * (L->nyq ? 2 : 1) * fused_hpitch(G.N) * (L->prec == WKE_F64 ? 16 : 8));
        if (G.fp_lds + stage <= FP_LDS_LIMIT) {
            G.fp_off_ph = G.fp_lds;
            G.fp_lds += stage;
        }
    }
}

// The fused 2D form also needs few slab fields, a chunking of the
// interpolation sum and its LDS within bounds, at the given width.
bool fused_width_ok(PlanLayout* L, Group& G, int wide, int mfma) {
    if (L->d != 2 || !fp_feasible(L, G, 0, true)) return false;
    for (const InstDev& I : L->inst)
        if (I.N == G.N && I.n_slab > FUSED_MAX_SLAB) return false;
    const int kind = G.colkind, w0 = G.fp_wide, m0 = G.fp_mfma;
    G.colkind = 2;
    G.fp_wide = wide;
    G.fp_mfma = mfma;
    update_fp(L, G);
    const bool ok = G.fp_threads > 0 && G.fp_nwp > 0 && G.fp_lds <= FP_LDS_LIMIT;
    G.colkind = kind;
    G.fp_wide = w0;
    G.fp_mfma = m0;
    update_fp(L, G);
    return ok;
}

bool fused_feasible(PlanLayout* L, Group& G, int mfma) {
    return fused_width_ok(L, G, 1, mfma) || fused_width_ok(L, G, 0, mfma);
}

// Split instance i's quadrature sum over n workgroups per column block.
void set_split(PlanLayout* L, int i, int n) {
    InstDev& I = L->inst[i];
    n = std::max(L->min_ig[i], std::min(n, L->max_ig[i]));
    I.items_per_ig = (I.n_items + n - 1) / n;
    I.n_ig = (I.n_items + I.items_per_ig - 1) / I.items_per_ig;
}

namespace {

// Whether item group ig's slab-field subset is all of the instance's slab
// fields in order (the fused kernel then needs no list).
bool subset_is_identity(const PlanLayout& L, int i, int ig) {
    const long long so = L.ig_sub[i][ig];
    const int n = L.inst[i].n_slab;
    if (L.sub[so] != n) return false;
    for (int q = 0; q < n; ++q)
        if (L.sub[so + 1 + q] != q) return false;
    return true;
}

// Rounds of the field-parallel column pass for instance i under its current
// split: each item group's items are taken in order, and a round closes when
// the next item's new distinct fields would not fit the workgroup (cap lane
// groups) or its weights the weight buffer.
void build_rounds(PlanLayout* L, int i, int cap, bool fused) {
    const InstDev& I = L->inst[i];
    const int S = I.S_item, U = I.U_item;
    const std::vector<int>& fid = L->fid[i];
    const std::vector<int>& frep = L->frep[i];
    std::vector<RoundDesc>& rounds = L->rounds[i];
    std::vector<FieldRef>& flds = L->flds[i];
    std::vector<int>& lidx = L->lidx[i];
    std::vector<int>& uofs = L->uofs[i];
    const std::vector<UnitPat>& pat = L->pats[i];
    rounds.clear();
    flds.clear();
    lidx.assign(I.n_shift, 0);
    uofs.assign(I.n_shift, 0);
    L->ig_r0[i].assign(I.n_ig, 0);
    L->ig_r1[i].assign(I.n_ig, 0);
    L->ig_f0[i].assign(I.n_ig, 0);
    L->ig_nfl[i].assign(I.n_ig, 0);
    L->ig_sub[i].assign(I.n_ig, 0);
    int ng = 0, ni = 0, nsub = 0;
    for (int ig = 0; ig < I.n_ig; ++ig) {
        const int it0 = ig * I.items_per_ig, it1 = std::min(I.n_items, it0 + I.items_per_ig);
        L->ig_r0[i][ig] = (int)rounds.size();
        L->ig_f0[i][ig] = (int)flds.size();
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
            for (int id : order) flds.push_back(FieldRef{frep[id], L->hid[i][frep[id]]});
            for (int ls = ia * S; ls < ib * S; ++ls) lidx[ls] = local[fid[ls]];
            // what the kernel reads: a, then b and c of each unit (an item
            // has exactly 1 + 2U shifts, with or without antipodal pairs)
            for (int it = ia; it < ib; ++it) {
                const int* li = lidx.data() + (long long)it * S;
                int* uo = uofs.data() + (long long)it * S;
                auto off = [&](int k) { return factor_offset(I.d, I.N, I.nyq_zero != 0, k); };
                uo[0] = off(li[0]);
                for (int u = 0; u < U && 2 + 2 * u < S; ++u) {
                    uo[1 + 2 * u] = off(li[pat[u].b]);
                    uo[2 + 2 * u] = off(li[pat[u].c]);
                }
            }
            ng = std::max(ng, (int)order.size());
            ni = std::max(ni, ib - ia);
            ia = ib;
        }
        L->ig_r1[i][ig] = (int)rounds.size();
        L->ig_nfl[i][ig] = (int)flds.size() - L->ig_f0[i][ig];
        if (fused) {
            // the slab fields of this item group, in order of first use; its
            // rounds' fields then name them by their place in the list
            const long long off = L->sub_off[i] + (long long)ig * (1 + I.n_slab);
            std::vector<int> list;
            for (size_t q = L->ig_f0[i][ig]; q < flds.size(); ++q) {
                auto at = std::find(list.begin(), list.end(), flds[q].y);
                if (at == list.end()) {
                    list.push_back(flds[q].y);
                    at = list.end() - 1;
                }
                flds[q].y = (int)(at - list.begin());
            }
            L->sub[off] = (int)list.size();
            std::copy(list.begin(), list.end(), L->sub.begin() + off + 1);
            L->ig_sub[i][ig] = (int)off;
            nsub = std::max(nsub, (int)list.size());
        }
    }
    L->fp_ng[i] = ng;
    L->fp_ni[i] = ni;
    L->rounds_fused[i] = fused ? 1 : 0;
    L->fp_ns[i] = fused ? nsub : I.n_slab;
}

}  // namespace

void layout_split(PlanLayout* L, Group& G) {
    // the rounds are built whenever the field-parallel forms apply, so that
    // their launch shapes can be judged from any current form
    const int half = G.colkind == 1 && G.fp_half && fp_feasible(L, G, 1) ? 1 : 0;
    const bool fused = G.colkind == 2;
    const int cap = fp_feasible(L, G, 0, fused) ? fp_field_cap(L, G.N, half, fused) : 0;
    G.hB.clear();
    for (int i = 0; i < L->batch; ++i) {
        if (L->inst[i].N != G.N) continue;
        InstDev& I = L->inst[i];
        const long long C = columns_of(I);
        const int gb = G.colkind >= 1 ? fp_columns(I.d) : g_slots_columns(L->prec, I.d, I.N);
        I.n_cb = (int)((C + gb - 1) / gb);
        if (cap > 0) build_rounds(L, i, cap, G.colkind == 2);
        for (int cb = 0; cb < I.n_cb; ++cb)
            for (int ig = 0; ig < I.n_ig; ++ig) {
                TaskB tb{i, cb, ig, 0, 0, 0, 0, 0};
                if (cap > 0 && G.colkind >= 1) {
                    tb.r0 = L->ig_r0[i][ig];
                    tb.r1 = L->ig_r1[i][ig];
                    tb.f0 = L->ig_f0[i][ig];
                    tb.nfl = L->ig_nfl[i][ig];
                    if (G.colkind == 2) tb.sub = subset_is_identity(*L, i, ig) ? -1 : L->ig_sub[i][ig];
                }
                G.hB.push_back(tb);
            }
    }
    update_fp(L, G);
}

bool launch_fits(const Group& G) {
    if (G.colkind == 0) return true;
    if (G.fp_threads <= 0 || G.fp_lds == 0 || G.fp_lds > FP_LDS_LIMIT) return false;
    return G.colkind != 2 || G.fp_nwp >= 1;
}

// ---------------------------------------------------------------------------
// Consistency check.
// ---------------------------------------------------------------------------
namespace {

struct Checker {
    std::string err;
    bool ok(bool cond, const char* fmt, long long a = 0, long long b = 0, long long c = 0) {
        if (!cond && err.empty()) {
            char buf[320];
            std::snprintf(buf, sizeof buf, fmt, a, b, c);
            err = buf;
        }
        return cond;
    }
};

bool within(long long off, long long len, long long size) { return off >= 0 && len >= 0 && off + len <= size; }

}  // namespace

std::string check_layout(const PlanLayout& L) {
    Checker k;
    const int B = L.batch;
    k.ok(B >= 1 && (int)L.inst.size() == B && (int)L.desc.size() == B, "batch %lld: descriptor lists", B);
    long long state = 0, npat = 0;
    for (const auto& pv : L.pats) npat += (long long)pv.size();
    for (int i = 0; i < B && k.err.empty(); ++i) {
        const InstDev& I = L.inst[i];
        const long long np = I.n_pts;
        k.ok(I.off_state == state && I.off_spec0 == state, "instance %lld: packed offset %lld", i, I.off_state);
        state += np;
        k.ok(within(I.off_state, np, (long long)L.total_elems), "instance %lld: state range", i);
        k.ok(within(I.off_spec0, np, L.n_spec0), "instance %lld: spectrum range", i);
        k.ok(within(I.off_nodes, 2LL * I.Nr + (I.d + 1LL) * (I.Ns + I.Nsig), L.n_nodes), "instance %lld: nodes", i);
        k.ok(within(I.off_ph, (long long)(I.n_shift + I.nyq_zero) * I.d * I.N, L.n_ph), "instance %lld: phase rows", i);
        k.ok(within(I.off_unit, I.n_unit, L.n_unit), "instance %lld: unit weights", i);
        k.ok(I.n_shift == I.n_items * I.S_item && I.n_unit == I.n_items * I.U_item, "instance %lld: counts", i);
        k.ok(within(L.pat_off[i], I.U_item, npat), "instance %lld: unit-pattern offset", i);
        k.ok((int)L.pats[i].size() == I.U_item && I.U_item >= 1, "instance %lld: unit patterns %lld", i, I.U_item);
        for (const UnitPat& u : L.pats[i])
            k.ok(u.b >= 1 && u.b < I.S_item && u.c >= 1 && u.c < I.S_item && u.p3 >= 0 && u.p3 < I.Nsig &&
                     u.p3b < I.Nsig, "instance %lld: unit pattern (%lld, %lld)", i, u.b, u.c);
        k.ok(L.tw_off.count(I.N) && I.off_tw == L.tw_off.at(I.N) && within(I.off_tw, I.N, L.n_tw),
             "instance %lld: twiddles", i);
        k.ok(I.counter_off >= 0 && I.counter_off + (I.d == 2 ? I.N : (long long)I.N * I.N) <= L.n_counters,
             "instance %lld: arrival counters", i);
        k.ok(I.n_ig >= L.min_ig[i] && I.n_ig <= L.max_ig[i] && I.items_per_ig >= 1 &&
                 (long long)I.n_ig * I.items_per_ig >= I.n_items && (I.n_ig - 1LL) * I.items_per_ig < I.n_items,
             "instance %lld: item groups %lld x %lld", i, I.n_ig, I.items_per_ig);
        k.ok((long long)(I.items_per_ig) * (I.S_item + I.nyq_zero) <= HID_CAP,
             "instance %lld: %lld items' shifts exceed the staged table", i, I.items_per_ig);
        if (L.max_ig[i] > 1) k.ok(within(I.off_part, (long long)L.max_ig[i] * np, L.n_part), "instance %lld: partials", i);
        if (L.hrep.empty()) continue;               // before the fields are laid out
        // the fields and the tables sized from them
        k.ok(I.n_slab == (int)L.hrep[i].size() && I.n_slab >= 1, "instance %lld: slab fields %lld", i, I.n_slab);
        k.ok(within(I.off_G, (long long)I.n_slab * np, L.n_G), "instance %lld: slab-field workspace", i);
        k.ok(within(I.off_hrep, I.n_slab, L.n_hrep), "instance %lld: slab-field representatives", i);
        k.ok(within(I.off_hid, I.n_shift + (long long)I.nyq_zero * (1 + I.n_items), L.n_hid),
             "instance %lld: per-shift tables", i);
        k.ok(within(I.off_rounds, I.n_items, L.n_rounds), "instance %lld: round table", i);
        if (I.d == 2) k.ok(within(I.off_kt, 2LL * I.n_slab * I.N, L.n_kt), "instance %lld: interpolation table (%lld of %lld)",
                           i, I.off_kt + 2LL * I.n_slab * I.N, L.n_kt);
        k.ok((int)L.hid[i].size() == I.n_shift + I.nyq_zero && (int)L.fid[i].size() == I.n_shift + I.nyq_zero,
             "instance %lld: shift maps", i);
        for (int h : L.hid[i]) k.ok(h >= 0 && h < I.n_slab, "instance %lld: slab field %lld", i, h);
        for (int r : L.hrep[i]) k.ok(r >= 0 && r < I.n_shift + I.nyq_zero, "instance %lld: representative %lld", i, r);
        for (int f : L.fid[i]) k.ok(f >= 0 && f < (int)L.frep[i].size(), "instance %lld: field id %lld", i, f);
        // rounds of the current split
        if (L.rounds[i].empty()) continue;
        k.ok((int)L.ig_r0[i].size() == I.n_ig && (int)L.ig_r1[i].size() == I.n_ig, "instance %lld: round index", i);
        k.ok((int)L.rounds[i].size() <= I.n_items, "instance %lld: %lld rounds", i, (long long)L.rounds[i].size());
        k.ok((long long)L.flds[i].size() <= L.n_hid - I.off_hid, "instance %lld: round fields %lld", i,
             (long long)L.flds[i].size());
        k.ok((int)L.lidx[i].size() == I.n_shift, "instance %lld: local field table", i);
        int item = 0;
        for (int ig = 0; ig < I.n_ig && k.err.empty(); ++ig) {
            const int it0 = ig * I.items_per_ig, it1 = std::min(I.n_items, it0 + I.items_per_ig);
            k.ok(L.ig_r0[i][ig] <= L.ig_r1[i][ig] && L.ig_r1[i][ig] <= (int)L.rounds[i].size(),
                 "instance %lld: item group %lld rounds", i, ig);
            k.ok(L.ig_f0[i][ig] >= 0 && L.ig_nfl[i][ig] <= HID_CAP &&
                     L.ig_f0[i][ig] + L.ig_nfl[i][ig] <= (int)L.flds[i].size(),
                 "instance %lld: item group %lld fields", i, ig);
            for (int r = L.ig_r0[i][ig]; r < L.ig_r1[i][ig]; ++r) {
                const RoundDesc& R = L.rounds[i][r];
                k.ok(R.ia == item && R.ib > R.ia && R.ib <= it1 && R.ia >= it0, "instance %lld: round %lld items", i, r);
                item = R.ib;
                k.ok(R.foff >= L.ig_f0[i][ig] && R.foff + R.nf <= L.ig_f0[i][ig] + L.ig_nfl[i][ig],
                     "instance %lld: round %lld field range", i, r);
                k.ok((R.ib - R.ia) * I.U_item <= FP_MAX_GROUPS, "instance %lld: round %lld weights", i, r);
                for (int ls = R.ia * I.S_item; ls < R.ib * I.S_item; ++ls) {
                    const int lf = L.lidx[i][ls];
                    k.ok(lf >= 0 && lf < R.nf, "instance %lld: shift %lld local field %lld", i, ls, lf);
                    if (lf >= 0 && lf < R.nf) {
                        const FieldRef& fr = L.flds[i][R.foff + lf];
                        int slab = fr.y;
                        if (L.rounds_fused[i]) {       // a place in the item group's subset
                            const long long so = L.ig_sub[i][ig];
                            const bool in = so >= 0 && so < L.n_sub && fr.y >= 0 && fr.y < L.sub[so];
                            k.ok(in, "instance %lld: shift %lld outside its slab-field subset", i, ls);
                            slab = in ? L.sub[so + 1 + fr.y] : -1;
                        }
                        k.ok(L.fid[i][fr.x] == L.fid[i][ls] && slab == L.hid[i][fr.x],
                             "instance %lld: shift %lld mapped to a different field", i, ls);
                    }
                }
                // the kernel's factor offsets: the pattern's fields, inside
                // the round's field blocks
                k.ok(1 + 2 * I.U_item == I.S_item && (int)L.uofs[i].size() == I.n_shift,
                     "instance %lld: factor offset table", i);
                const bool real = I.nyq_zero != 0;
                const long long lim = (long long)factor_offset(I.d, I.N, real, real ? 2 * ((R.nf + 1) / 2) : R.nf);
                for (int it = R.ia; it < R.ib && k.err.empty() && 1 + 2 * I.U_item == I.S_item; ++it) {
                    const int* li = L.lidx[i].data() + (long long)it * I.S_item;
                    const int* uo = L.uofs[i].data() + (long long)it * I.S_item;
                    bool same = uo[0] == factor_offset(I.d, I.N, real, li[0]);
                    for (int u = 0; u < I.U_item; ++u) {
                        const UnitPat& up = L.pats[i][u];
                        same = same && up.b > 0 && up.b < I.S_item && up.c > 0 && up.c < I.S_item &&
                               uo[1 + 2 * u] == factor_offset(I.d, I.N, real, li[up.b]) &&
                               uo[2 + 2 * u] == factor_offset(I.d, I.N, real, li[up.c]);
                    }
                    k.ok(same, "instance %lld: item %lld factor offsets differ from its fields", i, it);
                    for (int e = 0; e < I.S_item; ++e)
                        k.ok(uo[e] >= 0 && uo[e] < lim, "instance %lld: item %lld factor offset %lld outside the "
                             "round's field blocks", i, it, uo[e]);
                }
                for (int q = R.foff; q < R.foff + R.nf; ++q)
                    k.ok(L.flds[i][q].x >= 0 && L.flds[i][q].x < I.n_shift + I.nyq_zero && L.flds[i][q].y >= 0 &&
                             L.flds[i][q].y < I.n_slab, "instance %lld: round field %lld", i, q);
            }
            k.ok(item == it1, "instance %lld: item group %lld covers its items", i, ig);
            if (L.rounds_fused[i]) {
                const long long so = L.ig_sub[i][ig];
                k.ok(so >= L.sub_off[i] && so + 1 + I.n_slab <= L.sub_off[i] + (long long)L.max_ig[i] * (1 + I.n_slab) &&
                         so + 1 + I.n_slab <= L.n_sub, "instance %lld: item group %lld subset offset", i, ig);
                const int cnt = L.sub[so];
                k.ok(cnt >= 1 && cnt <= I.n_slab && cnt <= FUSED_MAX_SLAB && cnt <= L.fp_ns[i],
                     "instance %lld: item group %lld subset of %lld slab fields", i, ig, cnt);
                for (int q = 0; q < cnt && q < I.n_slab; ++q)
                    k.ok(L.sub[so + 1 + q] >= 0 && L.sub[so + 1 + q] < I.n_slab, "instance %lld: subset entry %lld",
                         i, L.sub[so + 1 + q]);
            }
        }
    }
    k.ok(state == (long long)L.total_elems && state == L.n_spec0, "packed length %lld", state);
    for (const Group& G : L.groups) {
        if (!k.err.empty()) break;
        for (const TaskA& t : G.hA) {
            k.ok(t.inst >= 0 && t.inst < B && L.inst[t.inst].N == G.N, "slab task of instance %lld", t.inst);
            if (t.inst < 0 || t.inst >= B) break;
            const InstDev& I = L.inst[t.inst];
            k.ok(t.j0 >= 0 && t.j0 < I.N && t.s_begin >= 0 && t.s_begin < t.s_end && t.s_end <= I.n_slab,
                 "slab task (%lld, %lld, %lld)", t.inst, t.j0, t.s_end);
        }
        k.ok(G.hA.size() <= G.maxA, "slab tasks %lld exceed the device list %lld", (long long)G.hA.size(),
             (long long)G.maxA);
        k.ok(G.hB.size() <= G.maxB, "column tasks %lld exceed the device list %lld", (long long)G.hB.size(),
             (long long)G.maxB);
        for (const TaskB& t : G.hB) {
            k.ok(t.inst >= 0 && t.inst < B, "column task of instance %lld", t.inst);
            if (t.inst < 0 || t.inst >= B) break;
            const InstDev& I = L.inst[t.inst];
            k.ok(I.N == G.N && t.cb >= 0 && t.cb < I.n_cb && t.ig >= 0 && t.ig < I.n_ig,
                 "column task (%lld, %lld, %lld)", t.inst, t.cb, t.ig);
            if (G.colkind >= 1)
                k.ok(t.r0 == L.ig_r0[t.inst][t.ig] && t.r1 == L.ig_r1[t.inst][t.ig] && t.nfl <= HID_CAP,
                     "column task (%lld, %lld): rounds", t.inst, t.ig);
            if (G.colkind == 2)
                k.ok(L.rounds_fused[t.inst] &&
                         (t.sub == L.ig_sub[t.inst][t.ig] || (t.sub == -1 && subset_is_identity(L, t.inst, t.ig))),
                     "column task (%lld, %lld): subset", t.inst, t.ig);
        }
        if (G.hB.empty()) continue;                 // column pass not laid out yet (plan creation in progress)
        if (G.colkind >= 1) {
            k.ok(G.fp_threads > 0 && G.fp_threads % 64 == 0 && G.fp_threads <= fp_max_threads(L.prec, G.N, G.colkind == 2, L.nyq != 0),
                 "field-parallel threads %lld",
                 G.fp_threads);
            k.ok(G.fp_lds > 0 && G.fp_lds <= FP_LDS_LIMIT, "field-parallel LDS %lld bytes", G.fp_lds);
            int ng = 0;
            for (int i = 0; i < B; ++i)
                if (L.inst[i].N == G.N) ng = std::max(ng, L.fp_ng[i]);
            const int blocks = L.nyq ? (ng + 1) / 2 : ng;
            Geometry g;
            geometry_of(L.prec, L.d, G.N, &g);
            k.ok((long long)blocks * fp_columns(L.d) * g.tpt <= G.fp_threads, "%lld field blocks need more lanes", blocks);
        }
        if (G.colkind == 2 && !G.fp_mfma)
            k.ok(G.fp_nwp >= 1 && G.fp_nwp * G.N <= G.fp_threads && (G.N / G.fp_nwp) % 8 == 0,
                 "fused chunks %lld", G.fp_nwp);
        if (G.colkind == 2 && G.fp_mfma)
            k.ok(G.fp_nwp >= 1 && (G.N / 4) % G.fp_nwp == 0 && G.N % 16 == 0, "matrix-core depth splits %lld",
                 G.fp_nwp);
        if (G.colkind == 2) {
            for (int i = 0; i < B; ++i)
                if (L.inst[i].N == G.N) k.ok(L.inst[i].n_slab <= FUSED_MAX_SLAB, "fused: %lld slab fields", L.inst[i].n_slab);
            k.ok(G.fp_off_h % 16 == 0 && G.fp_off_h < G.fp_lds, "fused LDS offset %lld", G.fp_off_h);
        }
        for (const TaskB& t : G.hF) {
            k.ok(t.inst >= 0 && t.inst < B, "forward task of instance %lld", t.inst);
        }
        // a single instance with one item group: the column pass may take
        // every task as the first one with its column block set to the
        // task's place in the list
        if (B == 1 && L.inst[0].n_ig == 1 && !G.hB.empty()) {
            const TaskB& t0 = G.hB[0];
            for (size_t q = 0; q < G.hB.size(); ++q) {
                const TaskB& t = G.hB[q];
                k.ok(t.inst == 0 && t.cb == (int)q && t.ig == 0 && t.r0 == t0.r0 && t.r1 == t0.r1 && t.f0 == t0.f0 &&
                         t.nfl == t0.nfl && t.sub == t0.sub,
                     "column task %lld differs from the first one but for its column block", (long long)q);
            }
        }
    }
    return k.err;
}

}  // namespace wke

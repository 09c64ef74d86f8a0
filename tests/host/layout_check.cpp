// CPU check of the plan layout (paper_2503_12805_amd/csrc/wke_layout.cpp),
// built with the address and undefined-behaviour sanitizers by
// tests/test_host_layout.py.  For many descriptors and batches, in both
// precisions and in the plain and the real form, it runs the layout steps
// the library runs at plan creation, then every column-pass form, width and
// work split the library can be switched to, and requires check_layout to
// find every offset, range, task and round consistent.  It also checks the
// table sizes against an independent count, and that check_layout reports
// an interpolation table sized before the slab-field count was known.
#include <cmath>
#include <cstdio>
#include <string>
#include <vector>

#include "wke_layout.hpp"

using namespace wke;

namespace {

// Quadrature nodes in the order the library's node kernel writes them
// (r, w_r, q-hat, w_s, sigma, w_sigma): Gauss-Legendre by Newton's method on
// the Legendre recurrence, midpoint angles (2i+1) pi / n, and the polyhedral
// designs in the library's vertex order.  Only the coincidences between
// shift vectors matter here, not the last bits.
void gauss_legendre(int n, double R, double* r, double* w) {
    for (int i = 0; i < n; ++i) {
        double x = std::cos(M_PI * (i + 0.75) / (n + 0.5)), dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = x;
            for (int k = 2; k <= n; ++k) {
                const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            if (n == 1) { p1 = x; p0 = 1.0; }
            dp = n * (p0 - x * p1) / (1.0 - x * x);
            const double dx = p1 / dp;
            x -= dx;
            if (std::fabs(dx) < 1e-16) break;
        }
        r[n - 1 - i] = 0.5 * R * (1.0 + x);
        w[n - 1 - i] = R / ((1.0 - x * x) * dp * dp);
    }
}

void sphere(int d, int rule, int n, double* P, double* W) {
    for (int i = 0; i < n; ++i) {
        if (d == 2) {
            P[2 * i] = std::cos((2.0 * i + 1.0) * M_PI / n);
            P[2 * i + 1] = std::sin((2.0 * i + 1.0) * M_PI / n);
            W[i] = 2.0 * M_PI / n;
            continue;
        }
        double v[3] = {0, 0, 0};
        if (rule == WKE_OCTAHEDRON) {
            v[i / 2] = (i & 1) ? -1.0 : 1.0;
        } else if (rule == WKE_CUBE) {
            const double q = 1.0 / std::sqrt(3.0);
            v[0] = (i & 4) ? -q : q;
            v[1] = (i & 2) ? -q : q;
            v[2] = (i & 1) ? -q : q;
        } else {
            const double phi = 0.5 * (1.0 + std::sqrt(5.0)), nr = std::sqrt(1.0 + phi * phi);
            const int cyc = i / 4;
            const double u[3] = {0.0, ((i >> 1) & 1) ? -1.0 : 1.0, (i & 1) ? -phi : phi};
            for (int a = 0; a < 3; ++a) v[(a + cyc) % 3] = u[a] / nr;
        }
        for (int a = 0; a < 3; ++a) P[3 * i + a] = v[a];
        W[i] = 4.0 * M_PI / n;
    }
}

std::vector<double> nodes_of(const PlanLayout& L) {
    std::vector<double> nd(std::max<long long>(1, L.n_nodes));
    for (const InstDev& I : L.inst) {
        double* r = nd.data() + I.off_nodes;
        double* wr = r + I.Nr;
        double* qh = wr + I.Nr;
        double* ws = qh + I.Ns * I.d;
        double* sg = ws + I.Ns;
        double* wsig = sg + I.Nsig * I.d;
        gauss_legendre(I.Nr, I.R, r, wr);
        sphere(I.d, I.rule, I.Ns, qh, ws);
        sphere(I.d, I.rule, I.Nsig, sg, wsig);
    }
    return nd;
}

int failures = 0, layouts = 0;

void expect(bool cond, const std::string& what) {
    if (!cond) {
        ++failures;
        std::printf("FAIL: %s\n", what.c_str());
    }
}

std::string name_of(const std::vector<wke_desc>& ds, int prec, int nyq) {
    char buf[160];
    std::snprintf(buf, sizeof buf, "batch %zu, first d=%d N=%d (%d,%d,%d), prec %d, real %d", ds.size(), ds[0].d,
                  ds[0].N, ds[0].N_r, ds[0].N_s, ds[0].N_sig, prec, nyq);
    return buf;
}

void run(const std::vector<wke_desc>& ds, int prec, int nyq) {
    const std::string nm = name_of(ds, prec, nyq);
    std::string err;
    if (validate_descs(ds.data(), (int)ds.size(), prec, &err) != WKE_OK) {
        expect(false, nm + ": descriptors refused: " + err);
        return;
    }
    PlanLayout L;
    layout_instances(&L, ds.data(), (int)ds.size(), prec, nyq);
    expect(check_layout(L).empty(), nm + ": instances: " + check_layout(L));
    const std::vector<double> nd = nodes_of(L);
    layout_fields(&L, nd.data());
    expect(check_layout(L).empty(), nm + ": fields: " + check_layout(L));
    // independent count of the tables sized from the slab fields
    long long kt = 0, G = 0;
    for (const InstDev& I : L.inst) {
        if (I.d == 2) kt += 2LL * (long long)L.hrep[&I - L.inst.data()].size() * I.N;
        G += (long long)L.hrep[&I - L.inst.data()].size() * I.n_pts;
    }
    expect(kt == L.n_kt && G == L.n_G, nm + ": table sizes");
    layout_tasks(&L);
    for (Group& g : L.groups) {                 // as at plan creation, checked after each group
        if (nyq && !g.colkind) continue;
        layout_split(&L, g);
        expect(check_layout(L).empty(), nm + ": group by group: " + check_layout(L));
    }
    if (nyq) {
        bool refused = false;
        for (const Group& g : L.groups) refused |= !g.colkind;
        if (refused) return;                    // the library refuses this plan
    }
    expect(check_layout(L).empty(), nm + ": tasks: " + check_layout(L));
    for (Group& g : L.groups) {
        if (nyq && !g.colkind) continue;        // the library refuses this plan
        // both slab-pass workgroup widths the autotuner can choose
        for (int alt = 0; alt <= (slab_alt_available(&L, g) ? 1 : 0); ++alt) {
            layout_slab_tasks(&L, g, alt);
            ++layouts;
            expect(check_layout(L).empty() && g.slab_alt == alt, nm + ": slab-pass width: " + check_layout(L));
        }
        layout_slab_tasks(&L, g, -1);
        int max_split = 1;
        for (int i = 0; i < L.batch; ++i)
            if (L.inst[i].N == g.N) max_split = std::max(max_split, L.max_ig[i]);
        for (int kind = nyq ? 1 : 0; kind <= 2; ++kind) {
            if (kind >= 1 && !fp_feasible(&L, g)) continue;
            if (kind == 2 && !fused_feasible(&L, g)) continue;
            for (int wide = 0; wide <= 3; ++wide) {    // 2, 3: the matrix-core fused form
                const int mfma = wide >> 1;
                if (mfma && kind != 2) continue;
                if (kind == 2 && !fused_width_ok(&L, g, wide & 1, mfma)) continue;
                for (int half = 0; half <= (kind == 1 ? 1 : 0); ++half) {
                    if (half && !fp_feasible(&L, g, 1)) continue;
                    int fitting = 0;
                    for (int n = 1; n <= max_split + 1; ++n) {
                        for (int i = 0; i < L.batch; ++i)
                            if (L.inst[i].N == g.N) set_split(&L, i, n);
                        g.colkind = kind;
                        g.fp_wide = wide & 1;
                        g.fp_mfma = mfma;
                        g.fp_half = half;
                        layout_split(&L, g);
                        if (!launch_fits(g)) continue;  // refused by the library
                        ++fitting;
                        ++layouts;
                        const std::string e = check_layout(L);
                        char buf[96];
                        std::snprintf(buf, sizeof buf, ": N=%d form %d wide %d half %d split %d: ", g.N, kind, wide,
                                      half, n);
                        expect(e.empty(), nm + buf + e);
                    }
                    char buf[96];
                    std::snprintf(buf, sizeof buf, ": N=%d form %d wide %d half %d fits no split", g.N, kind, wide, half);
                    expect(fitting > 0, nm + buf);
                }
            }
        }
        // back to the form and split the plan starts with
        for (int i = 0; i < L.batch; ++i)
            if (L.inst[i].N == g.N) set_split(&L, i, 1);
        g.colkind = fp_feasible(&L, g) ? 1 : 0;
        g.fp_wide = 0;
        g.fp_half = 0;
        g.fp_mfma = 0;
        layout_split(&L, g);
    }
    // an interpolation table sized before the slab-field counts were known
    // (every instance counted with no slab fields) must be reported
    bool any2d = false;
    for (const InstDev& I : L.inst) any2d |= I.d == 2;
    if (any2d) {
        PlanLayout bad = L;
        bad.n_kt = 0;
        for (InstDev& I : bad.inst) I.off_kt = 0;
        const std::string e = check_layout(bad);
        expect(e.find("interpolation table") != std::string::npos, nm + ": undersized interpolation table not reported");
    }
}

wke_desc D2(int N, double L, int nr, int ns, int nsig) { return wke_desc{2, N, L, 0.0, nr, ns, nsig, WKE_MIDPOINT}; }
wke_desc D3(int N, double L, int nr, int rule) {
    const int np = rule == WKE_OCTAHEDRON ? 6 : rule == WKE_CUBE ? 8 : 12;
    return wke_desc{3, N, L, 0.0, nr, np, np, rule};
}

}  // namespace

int main() {
    std::vector<std::vector<wke_desc>> cases;
    const int quads[][3] = {{2, 4, 2}, {4, 4, 4}, {1, 2, 6}, {3, 3, 3}, {8, 8, 6}, {64, 12, 12}, {1, 4, 4},
                            {1, 1, 65}, {1, 1, 1}, {2, 4, 4}, {16, 32, 32}};
    for (int N : {16, 32, 48, 64, 96, 128})
        for (const auto& q : quads) cases.push_back({D2(N, 10.0, q[0], q[1], q[2])});
    for (int N : {16, 32, 64})
        for (int rule : {WKE_OCTAHEDRON, WKE_CUBE, WKE_ICOSAHEDRON})
            for (int nr : {1, 2, 4, 32}) cases.push_back({D3(N, 12.0, nr, rule)});
    // the uneven 2D batch (16 each of N = 32, 48, 64, 96) and the 3D batch of 8
    std::vector<wke_desc> c4, c5, mixed;
    for (int N : {32, 48, 64, 96})
        for (int k = 0; k < 16; ++k) c4.push_back(D2(N, 10.0, 4, 4, 4));
    for (int k = 0; k < 8; ++k) c5.push_back(D3(64, 12.0, 4, WKE_CUBE));
    mixed = {D2(32, 10.0, 4, 4, 4), D2(64, 6.6, 64, 12, 12), D2(48, 10.0, 2, 3, 3), D2(32, 8.0, 8, 8, 6)};
    cases.push_back(c4);
    cases.push_back(c5);
    cases.push_back(mixed);
    for (const auto& ds : cases)
        for (int prec = 0; prec <= 1; ++prec)
            for (int nyq = 0; nyq <= 1; ++nyq) run(ds, prec, nyq);
    {
        // The float fused form's lanes beyond one pass of nwp x N take a
        // share of the slab fields each.  The GPU form-agreement test's 2D
        // N = 48 (4,4,4) float case must exercise the uneven case: more than
        // one share, shares that split wavefronts, and a slab-field count
        // the shares do not divide.
        const std::vector<wke_desc> ds = {D2(48, 10.0, 4, 4, 4)};
        PlanLayout L;
        layout_instances(&L, ds.data(), 1, 1, 0);
        const std::vector<double> nd = nodes_of(L);
        layout_fields(&L, nd.data());
        layout_tasks(&L);
        Group& g = L.groups[0];
        g.colkind = 2;
        g.fp_mfma = 0;
        layout_split(&L, g);
        const int pass = g.fp_nwp * g.N, nsh = pass > 0 ? g.fp_threads / pass : 0, ns = L.inst[0].n_slab;
        std::printf("fused float N=48: %d lanes, %d chunks, %d shares of %d lanes, %d slab fields\n", g.fp_threads,
                    g.fp_nwp, nsh, pass, ns);
        expect(nsh > 1 && pass % 64 != 0 && ns % nsh != 0, "fused float N=48 shares are not the uneven case");
    }
    std::printf("%d layouts checked, %d failures\n", layouts, failures);
    if (failures == 0) std::printf("all layouts consistent\n");
    return failures == 0 ? 0 : 1;
}

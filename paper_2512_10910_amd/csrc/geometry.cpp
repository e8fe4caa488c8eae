// Host geometry for the partitioned network expansion: validation of the
// network definition (Sec. II.A), enumeration of the retained loop terms
// (Sec. III.A-B: excited-bond configurations of degree <= K without dangling
// excitations), per-class contraction plans and the FP64 combine tables.
#include "geometry.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <functional>
#include <map>
#include <numeric>
#include <set>

namespace pne {

namespace {

constexpr size_t kMaxListed = size_t(1) << 24;  // cluster entries over all listed configurations

uint64_t mix(uint64_t h, uint64_t v) {
    h ^= v + 0x9e3779b97f4a7c15ULL + (h << 6) + (h >> 2);
    return h * 0xff51afd7ed558ccdULL;
}

}  // namespace

bool Geometry::same_as(const Geometry &o) const {
    return n_sites == o.n_sites && n_bonds == o.n_bonds && n_open == o.n_open && rank == o.rank &&
           dim == o.dim && bu == o.bu && bul == o.bul && bv == o.bv && bvl == o.bvl &&
           open_site == o.open_site && open_slot == o.open_slot && part_off == o.part_off &&
           part_bond == o.part_bond && subs == o.subs;
}

namespace {

uint64_t geometry_hash(const Geometry &g) {
    uint64_t h = 1469598103934665603ULL;
    h = mix(h, g.n_sites);
    h = mix(h, g.n_bonds);
    h = mix(h, g.n_open);
    for (int x : g.rank) h = mix(h, x);
    for (int x : g.dim) h = mix(h, x);
    for (int b = 0; b < g.n_bonds; ++b) {
        h = mix(h, g.bu[b]);
        h = mix(h, g.bul[b]);
        h = mix(h, g.bv[b]);
        h = mix(h, g.bvl[b]);
    }
    for (int k = 0; k < g.n_open; ++k) {
        h = mix(h, g.open_site[k]);
        h = mix(h, g.open_slot[k]);
    }
    if (g.n_parts() > 0) {
        h = mix(h, 0x70617274ULL);
        for (int x : g.part_off) h = mix(h, x);
        for (int x : g.part_bond) h = mix(h, x);
        for (const auto &sp : g.subs) {
            h = mix(h, 0x73756270ULL ^ sp.x);
            for (int x : sp.off) h = mix(h, x);
            for (int x : sp.bond) h = mix(h, x);
        }
    }
    return h;
}

}  // namespace

std::string set_partitions(Geometry *g, int n, const int32_t *begin, const int32_t *bond) {
    if (n < 0) return "negative partition count";
    if (n > 0 && (!begin || !bond)) return "partition arrays missing";
    if (n > kMaxParts) return "unsupported: more than 32 partitions";
    if (n > 0 && g->n_open > 0) return "unsupported: partitions on a network with open legs";
    std::vector<int> off{0}, bonds;
    std::vector<uint32_t> parts(g->n_bonds, 0u);
    if (n > 0 && begin[0] != 0) return "partition offsets must start at 0";
    for (int p = 0; p < n; ++p) {
        if (begin[p + 1] <= begin[p]) return "a partition transects no bond";
        for (int k = begin[p]; k < begin[p + 1]; ++k) {
            int b = bond[k];
            if (b < 0 || b >= g->n_bonds) return "partition bond out of range";
            if (parts[b] & (1u << p)) return "bond listed twice in one partition";
            parts[b] |= 1u << p;
            bonds.push_back(b);
        }
        off.push_back((int)bonds.size());
    }
    g->part_off = std::move(off);
    g->part_bond = std::move(bonds);
    if (n > 0) g->bond_parts = std::move(parts);
    else g->bond_parts.clear();
    g->subs.clear();
    g->hash = geometry_hash(*g);
    return "";
}

std::string set_subpartitions(Geometry *g, uint32_t x, int n, const int32_t *begin, const int32_t *bond) {
    const int np = g->n_parts();
    if (np == 0) return "no partitions to refine";
    const uint32_t full = np == 32 ? 0xffffffffu : ((1u << np) - 1u);
    if (x == 0 || (x & ~full)) return "subset is empty or names a partition that does not exist";
    if (n < 0) return "negative sub-partition count";
    if (n > kMaxParts) return "unsupported: more than 32 sub-partitions";
    if (n > 0 && (!begin || !bond)) return "sub-partition arrays missing";
    if (n > 0 && begin[0] != 0) return "sub-partition offsets must start at 0";
    Geometry::SubParts sp;
    sp.x = x;
    for (int p = 0; p < n; ++p) {
        if (begin[p + 1] <= begin[p]) return "a sub-partition transects no bond";
        std::vector<char> seen(g->n_bonds, 0);
        for (int k = begin[p]; k < begin[p + 1]; ++k) {
            int b = bond[k];
            if (b < 0 || b >= g->n_bonds) return "sub-partition bond out of range";
            if (seen[b]) return "bond listed twice in one sub-partition";
            seen[b] = 1;
            sp.bond.push_back(b);
        }
        sp.off.push_back((int)sp.bond.size());
    }
    auto it = std::find_if(g->subs.begin(), g->subs.end(), [&](const Geometry::SubParts &e) { return e.x == x; });
    if (it != g->subs.end()) g->subs.erase(it);
    if (n > 0) {
        g->subs.push_back(std::move(sp));
        std::sort(g->subs.begin(), g->subs.end(),
                  [](const Geometry::SubParts &a, const Geometry::SubParts &b) { return a.x < b.x; });
    }
    g->hash = geometry_hash(*g);
    return "";
}

std::string build_geometry(const pne_network_desc *d, Geometry *g) {
    if (!d) return "null descriptor";
    if (d->n_sites <= 0) return "n_sites must be positive";
    if (d->n_bonds < 0 || d->n_open < 0) return "negative count";
    if (!d->site_rank || !d->leg_dim) return "site_rank/leg_dim missing";
    if (d->n_bonds > 0 && (!d->bond_site || !d->bond_leg)) return "bond arrays missing";
    if (d->n_open > 0 && !d->open_leg) return "open_leg missing";
    g->n_sites = d->n_sites;
    g->n_bonds = d->n_bonds;
    g->n_open = d->n_open;
    g->rank.assign(d->site_rank, d->site_rank + d->n_sites);
    g->slot_base.resize(g->n_sites + 1);
    int64_t nslots = 0;
    for (int s = 0; s < g->n_sites; ++s) {
        int r = g->rank[s];
        if (r < 1 || r > kMaxRank) return "site rank must be in [1, 8]";
        g->slot_base[s] = (int)nslots;
        nslots += r;
    }
    g->slot_base[g->n_sites] = (int)nslots;
    g->dim.assign(d->leg_dim, d->leg_dim + nslots);
    for (int s = 0; s < g->n_sites; ++s) {
        int64_t size = 1;
        for (int l = 0; l < g->rank[s]; ++l) {
            int dd = g->dim[g->slot(s, l)];
            if (dd < 1 || dd > kMaxDim) return "leg dimension must be in [1, 16]";
            size *= dd;
        }
        if (size > (1 << 20)) return "site tensor too large";
    }
    g->partner.assign(nslots, -1);
    g->is_open.assign(nslots, 0);
    g->bu.resize(g->n_bonds);
    g->bul.resize(g->n_bonds);
    g->bv.resize(g->n_bonds);
    g->bvl.resize(g->n_bonds);
    for (int b = 0; b < g->n_bonds; ++b) {
        int u = d->bond_site[2 * b], v = d->bond_site[2 * b + 1];
        int lu = d->bond_leg[2 * b], lv = d->bond_leg[2 * b + 1];
        if (u < 0 || u >= g->n_sites || v < 0 || v >= g->n_sites) return "bond site out of range";
        if (u == v) return "bond joins a site to itself";
        if (lu < 0 || lu >= g->rank[u] || lv < 0 || lv >= g->rank[v]) return "bond leg out of range";
        int su = g->slot(u, lu), sv = g->slot(v, lv);
        if (g->partner[su] >= 0 || g->partner[sv] >= 0) return "leg used twice";
        if (g->dim[su] != g->dim[sv]) return "bond dimension mismatch";
        g->partner[su] = sv;
        g->partner[sv] = su;
        g->bu[b] = u;
        g->bul[b] = lu;
        g->bv[b] = v;
        g->bvl[b] = lv;
    }
    g->open_site.resize(g->n_open);
    g->open_slot.resize(g->n_open);
    for (int k = 0; k < g->n_open; ++k) {
        int s = d->open_leg[2 * k], l = d->open_leg[2 * k + 1];
        if (s < 0 || s >= g->n_sites || l < 0 || l >= g->rank[s]) return "open leg out of range";
        int sl = g->slot(s, l);
        if (g->partner[sl] >= 0) return "leg used twice";
        g->partner[sl] = sl;  // reflection
        g->is_open[sl] = 1;
        g->open_site[k] = s;
        g->open_slot[k] = l;
        if (std::find(g->open_sites.begin(), g->open_sites.end(), s) == g->open_sites.end())
            g->open_sites.push_back(s);
    }
    for (int64_t sl = 0; sl < nslots; ++sl)
        if (g->partner[sl] < 0) return "a leg is neither bonded nor open";
    g->hash = geometry_hash(*g);
    return "";
}

// ----------------------------------------------------------------------------
// enumeration: Redelmeier's untried-set scheme on the line graph, rooted at
// every bond in turn with only larger bonds admitted, so each connected set
// appears once.  A branch stops when the remaining budget cannot repair its
// degree-1 sites (a new bond touches at most two sites).

namespace {

struct Enum {
    const Geometry &g;
    int K;
    std::vector<int> inc_ptr, inc;   // site -> incident bonds
    std::vector<char> exempt;        // sites with open legs
    std::vector<int> deg;
    std::vector<char> seen;
    std::vector<char> excitable;
    std::vector<int> cur;
    int loose = 0;                   // non-exempt sites of degree 1
    int root = 0;
    ClusterList *out;

    Enum(const Geometry &g_, int K_, ClusterList *o, bool full) : g(g_), K(K_), out(o) {
        inc_ptr.assign(g.n_sites + 1, 0);
        for (int b = 0; b < g.n_bonds; ++b) {
            inc_ptr[g.bu[b] + 1]++;
            inc_ptr[g.bv[b] + 1]++;
        }
        for (int s = 0; s < g.n_sites; ++s) inc_ptr[s + 1] += inc_ptr[s];
        inc.assign(inc_ptr[g.n_sites], 0);
        std::vector<int> fill(inc_ptr.begin(), inc_ptr.end() - 1);
        for (int b = 0; b < g.n_bonds; ++b) {
            inc[fill[g.bu[b]]++] = b;
            inc[fill[g.bv[b]]++] = b;
        }
        // the dangling rule exempts sites with open legs, and every site when
        // the complete expansion is wanted
        exempt.assign(g.n_sites, full ? 1 : 0);
        for (int s : g.open_site) exempt[s] = 1;
        deg.assign(g.n_sites, 0);
        seen.assign(g.n_bonds, 0);
        // a bond of dimension 1 has P = I and Q = 0: it is never excited
        excitable.assign(g.n_bonds, 0);
        for (int b = 0; b < g.n_bonds; ++b) excitable[b] = g.dim[g.slot(g.bu[b], g.bul[b])] > 1;
    }

    void touch(int s, int delta) {
        int before = deg[s];
        deg[s] += delta;
        if (exempt[s]) return;
        loose -= (before == 1);
        loose += (deg[s] == 1);
    }

    void push(int b) {
        cur.push_back(b);
        touch(g.bu[b], +1);
        touch(g.bv[b], +1);
    }
    void pop() {
        int b = cur.back();
        cur.pop_back();
        touch(g.bu[b], -1);
        touch(g.bv[b], -1);
    }

    void emit() {
        size_t at = out->bonds.size();
        out->bonds.insert(out->bonds.end(), cur.begin(), cur.end());
        std::sort(out->bonds.begin() + at, out->bonds.end());
        out->off.push_back((int)out->bonds.size());
    }

    template <class F>
    void neighbours(int b, F &&f) {
        const int ends[2] = {g.bu[b], g.bv[b]};
        for (int s : ends)
            for (int p = inc_ptr[s]; p < inc_ptr[s + 1]; ++p)
                if (inc[p] != b) f(inc[p]);
    }

    void grow(std::vector<int> untried) {
        if (loose == 0) emit();
        if ((int)cur.size() >= K) return;
        if (2 * (K - (int)cur.size()) < loose) return;
        while (!untried.empty()) {
            int b = untried.back();
            untried.pop_back();
            std::vector<int> next = untried;
            size_t mark_from = next.size();
            neighbours(b, [&](int nb) {
                if (nb > root && !seen[nb] && excitable[nb]) {
                    seen[nb] = 1;
                    next.push_back(nb);
                }
            });
            push(b);
            grow(next);
            pop();
            for (size_t i = mark_from; i < next.size(); ++i) seen[next[i]] = 0;
        }
    }

    void run() {
        for (root = 0; root < g.n_bonds; ++root) {
            if (!excitable[root]) continue;
            seen[root] = 1;
            std::vector<int> untried;
            neighbours(root, [&](int nb) {
                if (nb > root && !seen[nb] && excitable[nb]) {
                    seen[nb] = 1;
                    untried.push_back(nb);
                }
            });
            push(root);
            grow(untried);
            pop();
            for (int b : untried) seen[b] = 0;
            seen[root] = 0;
        }
    }
};

}  // namespace

void enumerate_clusters(const Geometry &g, int K, ClusterList *out, bool full) {
    out->off.assign(1, 0);
    out->bonds.clear();
    if (K <= 0 || g.n_bonds == 0) return;
    Enum e(g, K, out, full);
    e.run();
}

// ----------------------------------------------------------------------------
// contraction plans

namespace {

struct LocalCluster {
    std::vector<int> verts;                 // global site ids, ascending
    std::vector<int> bonds;                 // global bond ids, ascending (label = index)
    std::vector<std::vector<int>> vlegs;    // per local vertex: labels of its legs
    std::vector<int> label_dim;             // dims of labels (bonds: D-1, open: p)
    std::vector<int> label_open_index;      // global open-leg index for open labels, else -1
    std::vector<std::vector<int>> vslots;   // per local vertex: slot of each leg
};

LocalCluster localise(const Geometry &g, const int *bonds, int k) {
    LocalCluster lc;
    lc.bonds.assign(bonds, bonds + k);
    std::set<int> vs;
    for (int b : lc.bonds) {
        vs.insert(g.bu[b]);
        vs.insert(g.bv[b]);
    }
    lc.verts.assign(vs.begin(), vs.end());
    int nv = (int)lc.verts.size();
    lc.vlegs.assign(nv, {});
    lc.vslots.assign(nv, {});
    auto lidx = [&](int s) { return (int)(std::lower_bound(lc.verts.begin(), lc.verts.end(), s) - lc.verts.begin()); };
    for (int j = 0; j < k; ++j) {
        int b = lc.bonds[j];
        lc.label_dim.push_back(g.dim[g.slot(g.bu[b], g.bul[b])] - 1);
        lc.label_open_index.push_back(-1);
        int iu = lidx(g.bu[b]), iv = lidx(g.bv[b]);
        lc.vlegs[iu].push_back(j);
        lc.vslots[iu].push_back(g.bul[b]);
        lc.vlegs[iv].push_back(j);
        lc.vslots[iv].push_back(g.bvl[b]);
    }
    for (int kk = 0; kk < g.n_open; ++kk) {
        int s = g.open_site[kk];
        auto it = std::lower_bound(lc.verts.begin(), lc.verts.end(), s);
        if (it == lc.verts.end() || *it != s) continue;
        int iv = (int)(it - lc.verts.begin());
        int lab = (int)lc.label_dim.size();
        lc.label_dim.push_back(g.dim[g.slot(s, g.open_slot[kk])]);
        lc.label_open_index.push_back(kk);
        lc.vlegs[iv].push_back(lab);
        lc.vslots[iv].push_back(g.open_slot[kk]);
    }
    return lc;
}

// A cluster that is one simple cycle (every vertex with exactly two legs,
// all bond labels of one dimension, no open legs): the cycle walked from
// local vertex 0, as (vertex, leg towards the previous vertex, leg towards
// the next vertex) per position.  Empty for any other cluster.
std::vector<int> simple_cycle(const LocalCluster &lc) {
    const int nv = (int)lc.verts.size();
    if (nv < 2) return {};
    for (int v = 0; v < nv; ++v)
        if (lc.vlegs[v].size() != 2) return {};
    for (size_t l = 0; l < lc.label_dim.size(); ++l)
        if (lc.label_open_index[l] >= 0 || lc.label_dim[l] != lc.label_dim[0]) return {};
    std::vector<int> out;
    int v = 0, m_in = 1;  // enter vertex 0 through its leg 1, leave through leg 0
    std::vector<char> seen(nv, 0);
    for (int j = 0; j < nv; ++j) {
        if (seen[v]) return {};
        seen[v] = 1;
        const int m_out = 1 - m_in;
        out.push_back(v);
        out.push_back(m_in);
        out.push_back(m_out);
        const int lab = lc.vlegs[v][m_out];
        int nxt = -1, nm = -1;
        for (int u = 0; u < nv && nxt < 0; ++u) {
            if (u == v) continue;
            for (int m = 0; m < 2; ++m)
                if (lc.vlegs[u][m] == lab) {
                    nxt = u;
                    nm = m;
                }
        }
        if (nxt < 0) return {};
        v = nxt;
        m_in = nm;
    }
    if (v != 0 || m_in != 1) return {};  // must close on vertex 0's leg 1
    return out;
}

// Class key: structure of the cluster up to the labelling induced by sorted
// site and bond ids (translates on a lattice share it).
std::vector<int> class_key(const LocalCluster &lc, const Geometry &g) {
    std::vector<int> key;
    key.push_back((int)lc.verts.size());
    key.push_back((int)lc.label_dim.size());
    for (size_t v = 0; v < lc.vlegs.size(); ++v) {
        key.push_back((int)lc.vlegs[v].size());
        for (int lab : lc.vlegs[v]) key.push_back(lab);
    }
    for (int d : lc.label_dim) key.push_back(d);
    for (int o : lc.label_open_index) key.push_back(o >= 0 ? 1 + o : 0);
    (void)g;
    return key;
}

size_t prod_dims(const std::vector<int> &labs, const std::vector<int> &dims) {
    size_t p = 1;
    for (int l : labs) p *= (size_t)dims[l];
    return p;
}

// Greedy elimination order: each step absorbs the site that keeps the
// frontier smallest; every start site is tried and the cheapest kept.
std::vector<int> elimination_order(const LocalCluster &lc) {
    int nv = (int)lc.verts.size();
    std::vector<int> best;
    double best_cost = 1e300;
    size_t best_peak = SIZE_MAX;
    for (int start = 0; start < nv; ++start) {
        std::vector<int> order{start};
        std::vector<char> done(nv, 0);
        done[start] = 1;
        std::multiset<int> f;
        auto frontier_after = [&](const std::multiset<int> &cur, int v, std::multiset<int> *nxt, size_t *nsum) {
            std::multiset<int> r = cur;
            size_t s = 1;
            for (int lab : lc.vlegs[v]) {
                auto it = r.find(lab);
                if (it != r.end()) {
                    r.erase(it);
                    s *= (size_t)lc.label_dim[lab];
                } else {
                    r.insert(lab);
                }
            }
            if (nxt) *nxt = r;
            if (nsum) *nsum = s;
            size_t p = 1;
            for (int lab : r) p *= (size_t)lc.label_dim[lab];
            return p;
        };
        size_t ns = 1;
        size_t peak = frontier_after(f, start, &f, &ns);
        double cost = (double)peak;
        for (int step = 1; step < nv; ++step) {
            int pick = -1;
            size_t pick_f = SIZE_MAX;
            for (int v = 0; v < nv; ++v) {
                if (done[v]) continue;
                bool adj = false;
                for (int lab : lc.vlegs[v])
                    if (f.count(lab)) adj = true;
                if (!adj) continue;
                size_t fs = frontier_after(f, v, nullptr, nullptr);
                if (fs < pick_f) {
                    pick_f = fs;
                    pick = v;
                }
            }
            if (pick < 0) {  // disconnected (cannot happen for a cluster)
                for (int v = 0; v < nv; ++v)
                    if (!done[v]) { pick = v; break; }
            }
            std::multiset<int> nf;
            size_t fs = frontier_after(f, pick, &nf, &ns);
            cost += (double)fs * (double)ns;
            peak = std::max(peak, fs);
            f = nf;
            done[pick] = 1;
            order.push_back(pick);
        }
        if (peak < best_peak || (peak == best_peak && cost < best_cost)) {
            best_peak = peak;
            best_cost = cost;
            best = order;
        }
    }
    return best;
}

// Entry tables of one step (StepEnt): output entries o, then summed entries
// t, each in mixed radix with the last label fastest.  None (ent = -1) when
// a label has more than 16 values or the plan's tables would grow past
// kMaxStepEnts.
constexpr size_t kMaxStepEnts = size_t(1) << 22;

void step_entries(StepDesc *sd, std::vector<StepEnt> *ents) {
    sd->ent = -1;
    for (int k = 0; k < sd->n_ol; ++k)
        if (sd->out_dim[k] > 16) return;
    for (int k = 0; k < sd->n_sl; ++k)
        if (sd->sum_dim[k] > 16) return;
    if (ents->size() + (size_t)sd->n_out + (size_t)sd->n_sum > kMaxStepEnts) return;
    sd->ent = (int)ents->size();
    for (int o = 0; o < sd->n_out; ++o) {
        StepEnt e{0, 0u};
        int rem = o;
        for (int k = sd->n_ol - 1; k >= 0; --k) {
            const int dg = rem % sd->out_dim[k];
            rem /= sd->out_dim[k];
            e.f += dg * sd->out_fs[k];
            if (sd->out_xl[k] >= 0) e.xdig |= (uint32_t)dg << (4 * sd->out_xl[k]);
        }
        ents->push_back(e);
    }
    for (int t = 0; t < sd->n_sum; ++t) {
        StepEnt e{0, 0u};
        int rem = t;
        for (int k = sd->n_sl - 1; k >= 0; --k) {
            const int dg = rem % sd->sum_dim[k];
            rem /= sd->sum_dim[k];
            e.f += dg * sd->sum_fs[k];
            e.xdig |= (uint32_t)dg << (4 * sd->sum_xl[k]);
        }
        ents->push_back(e);
    }
}

bool build_steps(const LocalCluster &lc, const std::vector<int> &order, std::vector<StepDesc> *steps,
                 std::vector<StepEnt> *ents, size_t *max_f, int *out_size, std::string *err) {
    std::vector<int> F;  // labels of the running frontier, C order
    *max_f = 1;
    for (size_t si = 0; si < order.size(); ++si) {
        int v = order[si];
        const std::vector<int> &legs = lc.vlegs[v];
        StepDesc sd;
        std::memset(&sd, 0, sizeof sd);
        sd.vert = v;
        if ((int)legs.size() > kMaxLab) {
            *err = "unsupported: site with too many cluster legs";
            return false;
        }
        sd.n_xl = (int)legs.size();
        for (size_t m = 0; m < legs.size(); ++m) sd.x_excited[m] = lc.label_open_index[legs[m]] < 0 ? 1 : 0;
        // strides of F
        std::vector<int> fstride(F.size());
        {
            int st = 1;
            for (int i = (int)F.size() - 1; i >= 0; --i) {
                fstride[i] = st;
                st *= lc.label_dim[F[i]];
            }
        }
        auto fpos = [&](int lab) {
            for (size_t i = 0; i < F.size(); ++i)
                if (F[i] == lab) return (int)i;
            return -1;
        };
        std::vector<int> outl, outfs, outxl, suml, sumfs, sumxl;
        for (size_t i = 0; i < F.size(); ++i) {
            bool shared = std::find(legs.begin(), legs.end(), F[i]) != legs.end();
            if (!shared) {
                outl.push_back(F[i]);
                outfs.push_back(fstride[i]);
                outxl.push_back(-1);
            }
        }
        for (size_t m = 0; m < legs.size(); ++m) {
            int p = fpos(legs[m]);
            if (p >= 0) {
                suml.push_back(legs[m]);
                sumfs.push_back(fstride[p]);
                sumxl.push_back((int)m);
            } else {
                outl.push_back(legs[m]);
                outfs.push_back(0);
                outxl.push_back((int)m);
            }
        }
        if (si + 1 == order.size()) {
            // final output: open labels in global open-leg order
            std::vector<int> idx(outl.size());
            std::iota(idx.begin(), idx.end(), 0);
            for (int lab : outl)
                if (lc.label_open_index[lab] < 0) {
                    *err = "internal: bond label left in final frontier";
                    return false;
                }
            std::sort(idx.begin(), idx.end(), [&](int a, int b) {
                return lc.label_open_index[outl[a]] < lc.label_open_index[outl[b]];
            });
            std::vector<int> a2, b2, c2;
            for (int i : idx) {
                a2.push_back(outl[i]);
                b2.push_back(outfs[i]);
                c2.push_back(outxl[i]);
            }
            outl = a2;
            outfs = b2;
            outxl = c2;
        }
        if ((int)outl.size() > kMaxLab || (int)suml.size() > kMaxLab) {
            *err = "unsupported: cluster frontier has too many indices";
            return false;
        }
        sd.n_ol = (int)outl.size();
        sd.n_sl = (int)suml.size();
        size_t nout = 1, nsum = 1;
        for (size_t i = 0; i < outl.size(); ++i) {
            sd.out_dim[i] = lc.label_dim[outl[i]];
            sd.out_fs[i] = outfs[i];
            sd.out_xl[i] = outxl[i];
            nout *= (size_t)sd.out_dim[i];
        }
        for (size_t i = 0; i < suml.size(); ++i) {
            sd.sum_dim[i] = lc.label_dim[suml[i]];
            sd.sum_fs[i] = sumfs[i];
            sd.sum_xl[i] = sumxl[i];
            nsum *= (size_t)sd.sum_dim[i];
        }
        if (nout > (1u << 16)) {
            *err = "unsupported: cluster frontier too large";
            return false;
        }
        sd.n_out = (int)nout;
        sd.n_sum = (int)nsum;
        *max_f = std::max(*max_f, nout);
        step_entries(&sd, ents);
        steps->push_back(sd);
        F = outl;
    }
    *out_size = (int)prod_dims(F, lc.label_dim);
    return true;
}

}  // namespace

std::shared_ptr<GeoPlan> build_plan(const Geometry &g, int K, std::string *err, bool full) {
    auto plan = std::make_shared<GeoPlan>();
    plan->K = K;
    if (full) {
        if (g.n_open > 0 || g.n_parts() > 0) {
            *err = "unsupported: the complete-expansion mode takes closed networks without partitions";
            return nullptr;
        }
        if (g.n_bonds > kMaxFullBonds) {
            *err = "unsupported: the complete-expansion mode takes at most 20 bonds";
            return nullptr;
        }
    }
    if ((int)g.open_sites.size() > 2) {
        *err = "unsupported: more than two sites carry open legs";
        return nullptr;
    }
    // open legs of a site must be listed together and in slot order
    for (int k = 1; k < g.n_open; ++k) {
        if (g.open_site[k] == g.open_site[k - 1]) {
            if (g.open_slot[k] <= g.open_slot[k - 1]) {
                *err = "unsupported: open legs of a site not in slot order";
                return nullptr;
            }
        } else {
            for (int j = 0; j < k - 1; ++j)
                if (g.open_site[j] == g.open_site[k]) {
                    *err = "unsupported: open legs of a site not listed together";
                    return nullptr;
                }
        }
    }
    int pdim[2] = {1, 1};
    for (int k = 0; k < g.n_open; ++k) {
        int which = g.open_site[k] == g.open_sites[0] ? 0 : 1;
        pdim[which] *= g.dim[g.slot(g.open_site[k], g.open_slot[k])];
    }
    plan->open_a = g.open_sites.size() > 0 ? g.open_sites[0] : -1;
    plan->open_b = g.open_sites.size() > 1 ? g.open_sites[1] : -1;
    plan->pa = pdim[0];
    plan->pb = pdim[1];
    if (plan->pa * plan->pb > kMaxOpenOut) {
        *err = "unsupported: open output tensor too large";
        return nullptr;
    }

    ClusterList raw;
    enumerate_clusters(g, K, &raw, full);
    int nc = raw.count();

    // type and size, then order clusters by (type, size, discovery)
    std::vector<int> type(nc), size(nc);
    for (int c = 0; c < nc; ++c) {
        int t = 0;
        for (int p = raw.off[c]; p < raw.off[c + 1]; ++p) {
            int b = raw.bonds[p];
            for (int s : {g.bu[b], g.bv[b]}) {
                if (s == plan->open_a) t |= 1;
                if (s == plan->open_b) t |= 2;
            }
        }
        type[c] = t;
        size[c] = raw.off[c + 1] - raw.off[c];
    }
    std::vector<int> perm(nc);
    std::iota(perm.begin(), perm.end(), 0);
    std::stable_sort(perm.begin(), perm.end(), [&](int a, int b) {
        if (type[a] != type[b]) return type[a] < type[b];
        return size[a] < size[b];
    });
    ClusterList &cl = plan->clusters;
    cl.off.assign(1, 0);
    cl.bonds.clear();
    for (int i = 0; i < nc; ++i) {
        int c = perm[i];
        cl.bonds.insert(cl.bonds.end(), raw.bonds.begin() + raw.off[c], raw.bonds.begin() + raw.off[c + 1]);
        cl.off.push_back((int)cl.bonds.size());
        plan->ctype.push_back(type[c]);
        plan->csize.push_back(size[c]);
    }
    auto out_size_of_type = [&](int t) { return (t & 1 ? plan->pa : 1) * (t & 2 ? plan->pb : 1); };
    plan->w_off.resize(nc);
    int64_t w = 0;
    for (int c = 0; c < nc; ++c) {
        plan->w_off[c] = w;
        w += out_size_of_type(plan->ctype[c]);
    }
    plan->w_total = w;

    // buckets
    for (int c = 0; c < nc;) {
        int e = c;
        while (e < nc && plan->ctype[e] == plan->ctype[c] && plan->csize[e] == plan->csize[c]) ++e;
        plan->buckets.push_back(Bucket{plan->ctype[c], plan->csize[c], c, e, (int32_t)plan->w_off[c],
                                       out_size_of_type(plan->ctype[c])});
        c = e;
    }

    // classes and instances
    std::map<std::vector<int>, int> class_ids;
    plan->cls_of.resize(nc);
    plan->inst_of.resize(nc);
    for (int c = 0; c < nc; ++c) {
        int k = cl.off[c + 1] - cl.off[c];
        LocalCluster lc = localise(g, cl.bonds.data() + cl.off[c], k);
        if ((int)lc.verts.size() > kMaxVerts) {
            *err = "unsupported: cluster with too many sites";
            return nullptr;
        }
        std::vector<int> key = class_key(lc, g);
        auto it = class_ids.find(key);
        int cid;
        if (it == class_ids.end()) {
            cid = (int)plan->classes.size();
            class_ids.emplace(key, cid);
            std::vector<int> order = elimination_order(lc);
            ClassDesc cd;
            std::memset(&cd, 0, sizeof cd);
            cd.step_begin = (int)plan->steps.size();
            size_t mf = 1;
            int osz = 1;
            if (!build_steps(lc, order, &plan->steps, &plan->step_ents, &mf, &osz, err)) return nullptr;
            cd.n_steps = (int)plan->steps.size() - cd.step_begin;
            cd.max_sum = 0;
            for (int st = 0; st < cd.n_steps; ++st) {
                const StepDesc &sd = plan->steps[cd.step_begin + st];
                if (sd.ent < 0) {
                    cd.max_sum = 0;
                    break;
                }
                cd.max_sum = std::max(cd.max_sum, sd.n_sum);
            }
            cd.n_verts = (int)lc.verts.size();
            cd.max_f = (int)mf;
            int gsz = 1;
            while (gsz < 64 && (size_t)gsz < mf) gsz <<= 1;
            cd.group = gsz;
            cd.out_size = osz;
            if (osz != out_size_of_type(plan->ctype[c])) {
                *err = "internal: cluster output size mismatch";
                return nullptr;
            }
            plan->max_f = std::max(plan->max_f, mf);
            plan->classes.push_back(cd);
            plan->inst_cluster.emplace_back();
            plan->inst_site.emplace_back();
            plan->inst_slots.emplace_back();
            plan->loop_order.push_back(simple_cycle(lc));
            plan->loop_e.push_back(plan->loop_order.back().empty() ? 0 : lc.label_dim[0]);
        } else {
            cid = it->second;
        }
        plan->cls_of[c] = cid;
        plan->inst_of[c] = (int)plan->inst_cluster[cid].size();
        plan->inst_cluster[cid].push_back(c);
        for (size_t v = 0; v < lc.verts.size(); ++v) {
            plan->inst_site[cid].push_back(lc.verts[v]);
            uint32_t packed = 0;
            for (size_t m = 0; m < lc.vslots[v].size(); ++m) packed |= (uint32_t)lc.vslots[v][m] << (4 * m);
            plan->inst_slots[cid].push_back(packed);
        }
    }

    if (g.n_parts() > 0 || full) {
        // User partitions (Eqs. (4) / (7) with factorised multi-index projectors,
        // Eqs. (9) / (11)).  Dropping the residue removes exactly the
        // configurations that excite at least one bond of every partition
        // (with rank-1 P, Q_p = I - P_p is the sum of the terms with some bond
        // of p excited, Eq. (10)), so the retained configurations are the
        // vertex-disjoint cluster sets of degree <= K whose excited bonds miss
        // some partition.  They are listed one by one.
        // The complete-expansion mode lists every configuration of degree <= K
        // the same way, as its connected components, with no partition to miss.
        plan->listed = true;
        const int np = g.n_parts();
        const uint32_t all_parts = np == 32 ? 0xffffffffu : ((1u << np) - 1u);
        plan->cmask.assign(nc, 0u);
        std::vector<std::vector<int>> vs(nc);
        for (int c = 0; c < nc; ++c) {
            std::set<int> s2;
            for (int p = cl.off[c]; p < cl.off[c + 1]; ++p) {
                if (np > 0) plan->cmask[c] |= g.bond_parts[cl.bonds[p]];
                s2.insert(g.bu[cl.bonds[p]]);
                s2.insert(g.bv[cl.bonds[p]]);
            }
            vs[c].assign(s2.begin(), s2.end());
        }
        // Recursive partitioning: the term of first-level subset x, when x has
        // sub-partitions R_x, keeps only the configurations that leave some
        // sub-partition of R_x unexcited.  A configuration S then counts with
        //   c(S) = sum over non-empty x with no bond of x excited of
        //          (-1)^(|x|+1) [R_x absent, or S misses a sub-partition of R_x],
        // which is 1 for every S that misses a partition when nothing is refined.
        const int ns = (int)g.subs.size();
        std::vector<uint32_t> sfull(ns);
        std::vector<std::vector<uint32_t>> csub(ns, std::vector<uint32_t>(nc, 0u));
        for (int e = 0; e < ns; ++e) {
            const auto &sp = g.subs[e];
            const int nsp = (int)sp.off.size() - 1;
            sfull[e] = nsp == 32 ? 0xffffffffu : ((1u << nsp) - 1u);
            std::vector<uint32_t> bmask(g.n_bonds, 0u);
            for (int r = 0; r < nsp; ++r)
                for (int k = sp.off[r]; k < sp.off[r + 1]; ++k) bmask[sp.bond[k]] |= 1u << r;
            for (int c = 0; c < nc; ++c)
                for (int q = cl.off[c]; q < cl.off[c + 1]; ++q) csub[e][c] |= bmask[cl.bonds[q]];
        }
        auto coefficient = [&](uint32_t mask, const std::vector<uint32_t> &smask) {
            const uint32_t comp = all_parts & ~mask;
            int64_t coef = 0;
            for (uint32_t x = comp; x != 0; x = (x - 1) & comp) {
                int keep = 1;
                for (int e = 0; e < ns; ++e)
                    if (g.subs[e].x == x) keep = smask[e] != sfull[e];
                coef += (__builtin_popcount(x) & 1) ? keep : -keep;
            }
            return coef;
        };
        plan->coll_off.assign(1, 0);
        plan->coll_cl.clear();
        plan->coll_coef.clear();
        std::vector<int> chosen;
        std::vector<char> used(g.n_sites, 0);
        bool too_many = false;
        // depth-first over clusters in increasing index: each collection once
        std::function<void(int, int, uint32_t, const std::vector<uint32_t> &)> dfs =
            [&](int from, int deg, uint32_t mask, const std::vector<uint32_t> &smask) {
                std::vector<uint32_t> sm(ns);
                for (int c = from; c < nc && !too_many; ++c) {
                    if (deg + plan->csize[c] > K) continue;
                    bool free = true;
                    for (int v : vs[c]) free = free && !used[v];
                    if (!free) continue;
                    const uint32_t m = mask | plan->cmask[c];
                    if (np > 0 && m == all_parts) continue;  // no term keeps it, nor any superset
                    for (int e = 0; e < ns; ++e) sm[e] = smask[e] | csub[e][c];
                    chosen.push_back(c);
                    for (int v : vs[c]) used[v] = 1;
                    const int64_t coef = ns ? coefficient(m, sm) : 1;
                    if (coef != 0) {  // a zero coefficient may still extend to a non-zero one
                        plan->coll_cl.insert(plan->coll_cl.end(), chosen.begin(), chosen.end());
                        plan->coll_off.push_back((int)plan->coll_cl.size());
                        if (ns) plan->coll_coef.push_back((double)coef);
                        if (plan->coll_cl.size() > kMaxListed) too_many = true;
                    }
                    dfs(c + 1, deg + plan->csize[c], m, sm);
                    for (int v : vs[c]) used[v] = 0;
                    chosen.pop_back();
                }
            };
        dfs(0, 0, 0u, std::vector<uint32_t>(ns, 0u));
        if (too_many) {
            *err = "unsupported: too many retained configurations to list";
            return nullptr;
        }
        plan->n_configs = (int64_t)plan->coll_off.size() - 1;
        return plan;
    }

    // overlapping pairs within the budget (categories used by the sum)
    int min_size = nc ? *std::min_element(plan->csize.begin(), plan->csize.end()) : 0;
    std::vector<std::vector<int>> site_clusters(g.n_sites);
    std::vector<std::vector<int>> vset(nc);
    for (int c = 0; c < nc; ++c) {
        std::set<int> vs;
        for (int p = cl.off[c]; p < cl.off[c + 1]; ++p) {
            vs.insert(g.bu[cl.bonds[p]]);
            vs.insert(g.bv[cl.bonds[p]]);
        }
        vset[c].assign(vs.begin(), vs.end());
        if (plan->csize[c] + min_size <= K)
            for (int s : vset[c]) site_clusters[s].push_back(c);
    }
    auto wanted = [](int t1, int t2) {  // t1 >= t2
        return (t1 == 0 && t2 == 0) || (t2 == 0 && t1 != 0) || (t1 == 2 && t2 == 1);
    };
    std::map<std::pair<int, int>, std::vector<std::pair<int, int>>> cats;
    int64_t n_overlap_all = 0;
    for (int c = 0; c < nc; ++c) {
        if (plan->csize[c] + min_size > K) continue;
        std::set<int> partners;
        for (int s : vset[c])
            for (int c2 : site_clusters[s])
                if (c2 > c && plan->csize[c] + plan->csize[c2] <= K) partners.insert(c2);
        for (int c2 : partners) {
            int a = c, b = c2;
            if (plan->ctype[a] < plan->ctype[b]) std::swap(a, b);
            ++n_overlap_all;
            if (wanted(plan->ctype[a], plan->ctype[b])) cats[{plan->ctype[a], plan->ctype[b]}].push_back({a, b});
        }
    }
    for (auto &kv : cats) {
        PairCat pc;
        pc.t1 = kv.first.first;
        pc.t2 = kv.first.second;
        pc.begin = (int)plan->pair_a.size();
        for (auto &p : kv.second) {
            plan->pair_a.push_back(p.first);
            plan->pair_b.push_back(p.second);
        }
        pc.end = (int)plan->pair_a.size();
        plan->pair_cats.push_back(pc);
    }

    // collections of three or more clusters are outside the FP64 combine
    {
        std::vector<int> bysize(nc);
        std::iota(bysize.begin(), bysize.end(), 0);
        std::sort(bysize.begin(), bysize.end(), [&](int a, int b) { return plan->csize[a] < plan->csize[b]; });
        if (nc >= 3 && plan->csize[bysize[0]] + plan->csize[bysize[1]] + plan->csize[bysize[2]] <= K) {
            auto disjoint = [&](int a, int b) {
                const auto &x = vset[a], &y = vset[b];
                size_t i = 0, j = 0;
                while (i < x.size() && j < y.size()) {
                    if (x[i] == y[j]) return false;
                    if (x[i] < y[j]) ++i; else ++j;
                }
                return true;
            };
            for (int i = 0; i < nc; ++i) {
                int a = bysize[i];
                for (int j = i + 1; j < nc; ++j) {
                    int b = bysize[j];
                    if (plan->csize[a] + plan->csize[b] + min_size > K) break;
                    if (!disjoint(a, b)) continue;
                    for (int k2 = j + 1; k2 < nc; ++k2) {
                        int c3 = bysize[k2];
                        if (plan->csize[a] + plan->csize[b] + plan->csize[c3] > K) break;
                        if (disjoint(a, c3) && disjoint(b, c3)) {
                            *err = "unsupported: K admits configurations with three or more components";
                            return nullptr;
                        }
                    }
                }
            }
        }
    }

    // retained configurations: singles plus disjoint pairs within the budget
    {
        std::map<std::pair<int, int>, int64_t> cnt;  // (type, size) -> count
        for (int c = 0; c < nc; ++c) cnt[{plan->ctype[c], plan->csize[c]}]++;
        int64_t pairs = 0;
        for (auto &x : cnt)
            for (auto &y : cnt) {
                if (y.first < x.first) continue;
                if (x.first.second + y.first.second > K) continue;
                if ((x.first.first & y.first.first) != 0) continue;  // both touch the same open site
                if (x.first == y.first) pairs += x.second * (x.second - 1) / 2;
                else pairs += x.second * y.second;
            }
        int64_t overlap_relevant = 0;
        for (auto &kv : cats) overlap_relevant += (int64_t)kv.second.size();
        plan->n_configs = nc + pairs - overlap_relevant;
        (void)n_overlap_all;
    }
    return plan;
}

}  // namespace pne

// Host-side geometry: validation, cluster enumeration, contraction plans and
// combine tables.  Everything here depends only on the network's graph and
// leg dimensions (never on tensor values), so results are cached per
// (geometry, K) by the runtime.
#pragma once

#include <cstdint>
#include <memory>
#include <string>
#include <vector>

#include "pne.h"
#include "pne_internal.h"

namespace pne {

struct Geometry {
    int n_sites = 0, n_bonds = 0, n_open = 0;
    std::vector<int> rank;       // per site
    std::vector<int> slot_base;  // per site: first global slot
    std::vector<int> dim;        // per global slot
    std::vector<int> bu, bul, bv, bvl;
    std::vector<int> open_site, open_slot;
    std::vector<int> partner;    // per global slot: slot receiving its outgoing message
    std::vector<int> is_open;    // per global slot
    std::vector<int> open_sites; // distinct sites with open legs, by first open leg
    // user partitions (Sec. II.A-C): partition p transects bonds
    // part_bond[part_off[p] .. part_off[p+1]); empty when every bond is its
    // own partition under the degree cap only
    std::vector<int> part_off{0}, part_bond;
    std::vector<uint32_t> bond_parts;  // per bond: bit p set if partition p transects it
    // recursive partitioning (Sec. IV.A): the term of first-level subset x is
    // itself expanded over sub-partitions (same layout as part_off/part_bond)
    struct SubParts {
        uint32_t x = 0;
        std::vector<int> off{0}, bond;
        bool operator==(const SubParts &o) const { return x == o.x && off == o.off && bond == o.bond; }
    };
    std::vector<SubParts> subs;  // sorted by x
    uint64_t hash = 0;

    int n_parts() const { return (int)part_off.size() - 1; }

    int slot(int s, int l) const { return slot_base[s] + l; }
    bool same_as(const Geometry &o) const;
};

// Validate a descriptor and fill *g.  Returns an empty string or the reason.
std::string build_geometry(const pne_network_desc *desc, Geometry *g);

// Replace the partitions of *g (n = 0 clears them) and rehash.  Returns an
// empty string or the reason (prefixed "unsupported:" when valid but outside
// the implemented envelope).
std::string set_partitions(Geometry *g, int n, const int32_t *begin, const int32_t *bond);

// Give the first-level subset x (a non-empty set of the partitions) its own
// sub-partitions (n = 0 removes them) and rehash.
std::string set_subpartitions(Geometry *g, uint32_t x, int n, const int32_t *begin, const int32_t *bond);

struct ClusterList {
    std::vector<int> off{0};  // cluster c: bonds[off[c] .. off[c+1])
    std::vector<int> bonds;
    int count() const { return (int)off.size() - 1; }
};

// Every connected bond set of size <= K whose sites all have degree >= 2
// inside the set (sites with open legs: >= 1); with full, every connected
// bond set of size <= K.  Bonds of a cluster ascending.
void enumerate_clusters(const Geometry &g, int K, ClusterList *out, bool full = false);

struct GeoPlan {
    int K = 0;
    ClusterList clusters;             // ordered by (type, size, discovery)
    std::vector<int> ctype, csize;    // per cluster
    std::vector<int64_t> w_off;       // per cluster: offset of its weight values
    int64_t w_total = 0;
    std::vector<int> cls_of, inst_of; // per cluster: class and instance index

    std::vector<ClassDesc> classes;
    std::vector<StepDesc> steps;
    std::vector<StepEnt> step_ents;  // per step with tables: n_out + n_sum entries
    std::vector<std::vector<int>> inst_cluster;    // per class
    std::vector<std::vector<int>> inst_site;       // per class: n_inst * n_verts (local site ids)
    std::vector<std::vector<uint32_t>> inst_slots; // per class: n_inst * n_verts packed slots
    // per class, when the cluster is one simple cycle of legs of a single
    // dimension e (every site with exactly two cluster legs, no open leg):
    // for each cycle position, (local vertex, leg to the previous vertex,
    // leg to the next vertex); empty otherwise
    std::vector<std::vector<int>> loop_order;
    std::vector<int> loop_e;

    // with user partitions: every retained configuration listed as its
    // clusters coll_cl[coll_off[k] .. coll_off[k+1]) (pairwise vertex-disjoint,
    // total degree <= K, leaving at least one partition unexcited); empty
    // otherwise
    std::vector<uint32_t> cmask;      // per cluster: partitions it excites
    std::vector<int> coll_off, coll_cl;
    std::vector<double> coll_coef;    // per listed configuration, with sub-partitions; empty otherwise
    bool listed = false;

    std::vector<Bucket> buckets;
    std::vector<int> pair_a, pair_b;  // overlapping cluster pairs (|a|+|b| <= K)
    std::vector<PairCat> pair_cats;
    int open_a = -1, open_b = -1, pa = 1, pb = 1;
    int64_t n_configs = 0;
    size_t max_f = 1;
};

// Largest network the complete-expansion mode lists (2^20 - 1 configurations).
constexpr int kMaxFullBonds = 20;

// Build the plan; returns nullptr and sets *err (prefixed "unsupported:" when
// the geometry is valid but outside the implemented envelope).  full: every
// configuration of degree <= K, dangling ones included, each listed as its
// vertex-disjoint connected components (closed networks without partitions,
// at most kMaxFullBonds bonds).
std::shared_ptr<GeoPlan> build_plan(const Geometry &g, int K, std::string *err, bool full = false);

}  // namespace pne

// Host-only driver of the library's planner (validation, cluster
// enumeration, contraction plans, partition listing and coefficients), built
// with AddressSanitizer and UndefinedBehaviorSanitizer by the CPU tests.
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "geometry.h"

using namespace pne;

namespace {

// Lx x Ly open lattice, sites x + Lx y, legs (-x, +x, -y, +y) where present,
// bond dimension D, optional open leg of dimension 2 on site `open_site`.
struct Lattice {
    std::vector<int> rank, dims, bsite, bleg, oleg;
    std::vector<const double *> data;
    std::vector<double> dummy;
    pne_network_desc desc{};
    Lattice(int Lx, int Ly, int D, int open_site = -1) {
        const int n = Lx * Ly;
        std::vector<std::vector<int>> slot(n, std::vector<int>(4, -1));
        for (int s = 0; s < n; ++s) {
            const int x = s % Lx, y = s / Lx;
            int r = 0;
            if (x > 0) slot[s][0] = r++;
            if (x < Lx - 1) slot[s][1] = r++;
            if (y > 0) slot[s][2] = r++;
            if (y < Ly - 1) slot[s][3] = r++;
            int extra = s == open_site ? 1 : 0;
            rank.push_back(r + extra);
            for (int l = 0; l < r; ++l) dims.push_back(D);
            if (extra) {
                dims.push_back(2);
                oleg.push_back(s);
                oleg.push_back(r);
            }
        }
        for (int s = 0; s < n; ++s) {
            const int x = s % Lx, y = s / Lx;
            if (x < Lx - 1) {
                bsite.push_back(s), bsite.push_back(s + 1);
                bleg.push_back(slot[s][1]), bleg.push_back(slot[s + 1][0]);
            }
            if (y < Ly - 1) {
                bsite.push_back(s), bsite.push_back(s + Lx);
                bleg.push_back(slot[s][3]), bleg.push_back(slot[s + Lx][2]);
            }
        }
        dummy.assign(1, 0.0);
        data.assign(n, dummy.data());
        desc.n_sites = n;
        desc.n_bonds = (int)bsite.size() / 2;
        desc.n_open = (int)oleg.size() / 2;
        desc.site_rank = rank.data();
        desc.leg_dim = dims.data();
        desc.bond_site = bsite.data();
        desc.bond_leg = bleg.data();
        desc.open_leg = oleg.empty() ? nullptr : oleg.data();
        desc.site_data = data.data();
    }
};

int fails = 0;

void expect(bool ok, const char *what) {
    if (!ok) {
        std::printf("FAIL: %s\n", what);
        ++fails;
    }
}

}  // namespace

int main() {
    // plain plans of several shapes and degree caps
    for (int D : {2, 3, 4}) {
        Lattice L(4, 4, D);
        Geometry g;
        expect(build_geometry(&L.desc, &g).empty(), "4x4 geometry");
        for (int K : {0, 4, 6, 8}) {
            std::string err;
            auto p = build_plan(g, K, &err);
            expect(p != nullptr, "4x4 plan");
        }
    }
    {
        Lattice L(5, 4, 3, 7);  // one open leg
        Geometry g;
        expect(build_geometry(&L.desc, &g).empty(), "open geometry");
        std::string err;
        expect(build_plan(g, 6, &err) != nullptr, "open plan");
        int32_t begin[2] = {0, 1}, bond[1] = {0};
        expect(!set_partitions(&g, 1, begin, bond).empty(), "partitions on an open network refused");
    }
    // partitions, sub-partitions, listed collections with coefficients
    {
        Lattice L(3, 4, 3);
        Geometry g;
        expect(build_geometry(&L.desc, &g).empty(), "3x4 geometry");
        // two lines: bonds crossing x = 0|1 and y = 1|2
        std::vector<int32_t> begin{0}, bond;
        for (int b = 0; b < L.desc.n_bonds; ++b) {
            const int u = L.bsite[2 * b], v = L.bsite[2 * b + 1];
            if (v == u + 1 && u % 3 == 0) bond.push_back(b);
        }
        begin.push_back((int32_t)bond.size());
        for (int b = 0; b < L.desc.n_bonds; ++b) {
            const int u = L.bsite[2 * b], v = L.bsite[2 * b + 1];
            if (v == u + 3 && u / 3 == 1) bond.push_back(b);
        }
        begin.push_back((int32_t)bond.size());
        expect(set_partitions(&g, 2, begin.data(), bond.data()).empty(), "partitions");
        int32_t sb[3] = {0, 1, 2}, sbond[2] = {1, 4};
        expect(set_subpartitions(&g, 1u, 2, sb, sbond).empty(), "sub-partitions");
        for (int K : {4, 8, 17}) {
            std::string err;
            auto p = build_plan(g, K, &err);
            expect(p != nullptr && p->listed, "listed plan");
            if (p) expect(p->coll_coef.size() + 1 == p->coll_off.size(), "one coefficient per listed configuration");
        }
        expect(set_subpartitions(&g, 1u, 0, nullptr, nullptr).empty(), "remove sub-partitions");
        expect(!set_subpartitions(&g, 8u, 1, sb, sbond).empty(), "subset naming a missing partition refused");
        int32_t bad[1] = {99};
        expect(!set_subpartitions(&g, 1u, 1, sb, bad).empty(), "out-of-range sub-partition bond refused");
        expect(set_partitions(&g, 0, nullptr, nullptr).empty(), "clear partitions");
    }
    // complete-expansion mode: every connected bond set, every configuration listed
    {
        Lattice L(3, 3, 2);
        Geometry g;
        expect(build_geometry(&L.desc, &g).empty(), "3x3 geometry");
        for (int K : {1, 4, 12}) {
            std::string err;
            auto p = build_plan(g, K, &err, true);
            expect(p != nullptr && p->listed, "complete-expansion plan");
        }
        std::string err;
        auto p = build_plan(g, 12, &err, true);
        expect(p && p->n_configs == 4095, "2^12 - 1 configurations");
        Lattice B(5, 3, 2);  // 22 bonds
        Geometry gb;
        expect(build_geometry(&B.desc, &gb).empty(), "5x3 geometry");
        expect(build_plan(gb, 4, &err, true) == nullptr, "complete expansion above 20 bonds refused");
    }
    // malformed descriptors
    {
        Lattice L(3, 3, 2);
        Geometry g;
        L.bleg[0] = 7;
        expect(!build_geometry(&L.desc, &g).empty(), "leg out of range refused");
        Lattice M(3, 3, 2);
        M.dims[0] = 0;
        expect(!build_geometry(&M.desc, &g).empty(), "dimension 0 refused");
        expect(!build_geometry(nullptr, &g).empty(), "null descriptor refused");
    }
    std::printf("%s (%d failures)\n", fails ? "FAILED" : "ok", fails);
    return fails ? 1 : 0;
}

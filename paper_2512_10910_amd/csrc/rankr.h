// Internal interface of the rank-r (weight passing) expansion: the lattice
// description shared by the small- and large-bond-dimension kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "pne.h"

namespace pne {

constexpr int kRkSites = 16;  // sites per network
constexpr int kRkBonds = 32;  // bonds per network

struct RkGeo {
    int32_t n_sites, n_bonds, chi, Lx, Ly;
    int32_t rank[kRkSites];
    int32_t bu[kRkBonds], bul[kRkBonds], bv[kRkBonds], bvl[kRkBonds];
    int32_t leg_bond[kRkSites][4];  // bond on each leg slot (-1: none)
    int32_t dir_slot[kRkSites][4];  // slot of direction (-x, +x, -y, +y), -1 if absent
    int32_t toff[kRkSites + 1];     // packed offsets of the site tensors (chi^rank each)
};

// Per network: sum_t sgn[t] v_t exp(log_t - ref) over the n_terms (log, value)
// pairs in terms, plus the weight-passing log-scale, into res.
__global__ void k_rank_combine(const double *__restrict__ terms, const int8_t *__restrict__ sgn, int n_terms,
                               int n_nets, const double *__restrict__ log_all, pne_rank_result *__restrict__ res,
                               const int *__restrict__ sweeps_all, const int *__restrict__ status_all);

// HIP events between the phases of a profiled rank expansion: mark() after
// each phase's launches, read() once the stream has synchronised.
struct RankTimer {
    static constexpr int kMax = 6;
    hipEvent_t ev[kMax] = {};
    int n = 0;
    bool on;
    explicit RankTimer(bool enable) : on(enable) {}
    RankTimer(const RankTimer &) = delete;
    RankTimer &operator=(const RankTimer &) = delete;
    void mark(hipStream_t s) {
        if (!on || n >= kMax) return;
        if (hipEventCreate(&ev[n]) != hipSuccess) {
            on = false;
            return;
        }
        ++n;
        if (hipEventRecord(ev[n - 1], s) != hipSuccess) on = false;
    }
    // phase k (between marks k and k + 1) into out[k], k < nout; zeros if off
    void read(double *out, int nout) const {
        for (int k = 0; k < nout; ++k) {
            float ms = 0.0f;
            out[k] = (on && k + 1 < n && hipEventElapsedTime(&ms, ev[k], ev[k + 1]) == hipSuccess) ? ms : 0.0;
        }
    }
    ~RankTimer() {
        for (int k = 0; k < n; ++k) (void)hipEventDestroy(ev[k]);
    }
};

// Per-context phase times of the last profiled rank expansion (5 entries).
double *ctx_rank_times(pne_ctx *ctx);

// Largest bond dimension of the MFMA path, and whether (chi, Lx, Ly) is in
// its envelope: chi in {8, 16}, 2 <= Lx, chi^(Lx-1) a multiple of 16,
// chi^(Lx+1) <= 65536, Lx * Ly <= 16.
constexpr int kRkLargeChi = 16;
bool rank_large_supported(int chi, int Lx, int Ly);

// Weight passing and the expansion's terms for bond dimensions above 4
// (rankr_large.hip): same inputs and results as pne_rank_expand.  ops holds
// n_terms * n_bonds operator codes (0 whole weight, 1 P, 2 Q), sgn a sign per
// term.
pne_status rank_expand_large(pne_ctx *ctx, pne_network *const *nets, int32_t n, const RkGeo &geo,
                             const std::vector<int8_t> &ops, const std::vector<int8_t> &sgn, int n_terms,
                             const pne_rank_options *opt, pne_rank_result *results, RankTimer &timer);

}  // namespace pne

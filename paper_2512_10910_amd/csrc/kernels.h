// Launchers for the gfx950 kernels (defined in kernels.hip).  Plain C++
// signatures so the host runtime needs no device headers beyond hip_runtime.
#pragma once

#include <hip/hip_runtime.h>

#include "pne_internal.h"

namespace pne {

struct DeviceBatch {
    // tables
    const SiteRec *sites = nullptr;
    int n_sites = 0;
    const BpTile *tiles = nullptr;      // tiles swept by the per-sweep kernels
    int n_tiles = 0;
    int n_reg_tiles = 0;                // tiles[0, n_reg_tiles): register tiles (dynamic LDS reg_lds);
    int n_narrow_tiles = 0;             // then up to n_narrow_tiles the LDS tiles (bp_lds); then up
                                        // to n_wide_end register tiles of the wide shapes (rank 4 at
                                        // D = 5, 6; rank 6 at D = 3; wide_lds); the rest: rank 6 at
                                        // D = 4 (xwide_lds)
    const BpTile *all_tiles = nullptr;  // every tile (the fused kernel indexes it)
    const FusedNet *fused = nullptr;    // networks run by the persistent BP kernel: the large ones,
    int n_fused = 0;                    // then the n_fused_small small ones (two-wave blocks), then
    int n_fused_small = 0;              // the n_fused_big ones whose LDS needs the 256-VGPR kernel
    size_t fused_lds_small = 0;
    int n_fused_big = 0;
    size_t fused_lds_big = 0;
    const FusedGroup *fgroups = nullptr;
    const int *fsite_list = nullptr;
    size_t fused_lds = 0;
    int fused_regauge = 1;              // persistent blocks also build gauge + slices
    int reg_budget = 0;                 // persistent kernel: 0 two blocks per CU (128 VGPRs), 1 one (256)
    const int *tile_sites = nullptr;
    const int *init_sites = nullptr;    // sites whose messages k_init resets (non-persistent networks)
    int n_init_sites = 0;
    const int *init_nets = nullptr;     // networks whose state k_init resets (non-persistent networks)
    int n_init_nets = 0;
    size_t bp_lds = 0;             // dynamic LDS of the sweep kernel's LDS tiles
    size_t reg_lds = 0;            // ... of its register tiles (their raw outgoing messages)
    size_t wide_lds = 0;           // ... of the wide-shape register tiles
    size_t xwide_lds = 0;          // ... of the extra-wide (rank 6, D = 4) register tiles
    int n_wide_end = 0;            // tiles[n_wide_end, n_tiles): the extra-wide tiles
    // Where a sweep has wide tiles and others, the others (few, or short) run
    // on the context's side stream beside the wide launch: fork and join
    // events of the batch (null for a batch that must not create them).
    hipStream_t side = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
    NetState *state = nullptr;
    int n_nets = 0;
    // buffers
    double *msg0 = nullptr, *msg1 = nullptr;
    void *slices = nullptr;
    int precision = 0;
    double damping = 0.0;          // BP damping of the per-launch sweeps
    int bp_stall = 50;             // rounding-floor stop: sweeps without a new smallest residual (0: never)
    double bp_floor = 0.0;         // ... once that residual is at most this (100 * tol)
    double *site_log = nullptr;
    int *site_sign = nullptr;
    double *vac = nullptr;
    size_t regauge_lds = 0;
    const int *rg_tiles = nullptr;  // register-path tiles (indices into all_tiles) for the regauge
    int n_rg_tiles = 0;
    const int *rg_wide = nullptr;   // register tiles of one site whose shape holds 5..16 values
    int n_rg_wide = 0;              // per lane (indices into all_tiles), regauged by k_regauge_wide,
    static constexpr int kRgWideShapes = 4;  // grouped by shape (dim * 8 + rank)
    int n_rg_wide_groups = 0;
    int rg_wide_begin[kRgWideShapes + 1] = {};
    int rg_wide_shape[kRgWideShapes] = {};
    const int *rg_sites = nullptr;  // sites regauged one per block (open or mixed-dimension sites),
    int n_rg_sites = 0;             // sorted by size and launched in groups, each with its own LDS
    static constexpr int kRgGroups = 4;
    int n_rg_groups = 0;
    int rg_group_begin[kRgGroups + 1] = {};
    size_t rg_group_lds[kRgGroups] = {};
    // clusters
    const ClassDesc *classes = nullptr;
    const StepDesc *steps = nullptr;
    const StepEnt *step_ents = nullptr;
    const ClusterBlock *cblocks = nullptr;
    int n_cblocks = 0;
    static constexpr int kClKinds = 6;    // block ranges: frontier plans, cycles of leg
    int cl_kind_begin[kClKinds + 1] = {}; // dimension 2..5, scalar products
    const PlanNet *pnets = nullptr;       // per plan: its networks' slice and weight bases
    size_t cluster_lds = 0;
    double *w = nullptr;
    int64_t n_slice_elems = 0;  // extents the checked build tests cluster indices against
    int64_t n_w = 0;
    int n_step_ents = 0;
    // combine
    const CombineRec *crec = nullptr;
    const int *combine_nets = nullptr;   // networks summed by the combine launch
    int n_combine = 0;
    const GeoRec *geos = nullptr;
    const Bucket *buckets = nullptr;
    const int *pair_a = nullptr, *pair_b = nullptr;
    const PairCat *pair_cats = nullptr;
    const int *coll_off = nullptr, *coll_cl = nullptr;  // listed configurations (user partitions)
    const double *coll_coef = nullptr;                   // their coefficients (recursive partitioning)
    NetResult *results = nullptr;
    double *open_out = nullptr;  // open networks' output tensors (CombineRec::open_off)
};

// kernel identifiers for per-kernel timing (KID_GAUGE stays as a slot: the
// gauge is built inside the regauge kernels and has no launch of its own)
enum KernelId { KID_INIT = 0, KID_SWEEP, KID_CLOSE, KID_FUSED, KID_GAUGE, KID_REGAUGE, KID_CLUSTERS, KID_COMBINE, KID_COUNT };

// threads per BP tile and dynamic LDS (doubles) of one BP tile
int bp_tile_threads();
// sites per tile on the register path for uniform leg dimension D and rank R (0: LDS path)
// Networks of at most this many sites run in persistent blocks of 128
// threads (two waves) instead of 512.
constexpr int kPSmallSites = 64;  // default threshold (pne_options.small_sites)
int bp_reg_sites_per_tile(int D, int R);
// sites per register tile of the per-launch sweep (0: LDS path); a superset
// of the shapes bp_reg_sites_per_tile accepts
int bp_sweep_reg_sites_per_tile(int D, int R);
bool bp_sweep_xwide(int D, int R);
size_t bp_tile_lds_doubles(int n_sites, int size, int n_os, int last_dim, int max_dim);

hipError_t launch_init(const DeviceBatch &b, hipStream_t s);
hipError_t launch_sweep(const DeviceBatch &b, int k, double tol, int max_iter, hipStream_t s);
hipError_t launch_close(const DeviceBatch &b, int k_last, double tol, hipStream_t s);
hipError_t launch_fused(const DeviceBatch &b, double tol, int max_iter, hipStream_t s);
// doubles of dynamic LDS of a persistent block and its per-wave scratch
size_t bp_persistent_lds_doubles(int msg_size, int n_sites, int scratch_per_wave, int n_buffers, bool small);
int bp_persistent_scratch(int spw, int rank, int dim, int nt);
int bp_persistent_tiles_in_flight(int dim, int rank);
// shapes whose tiles in flight (1 or 2) a batch may choose
bool bp_persistent_tiles_tunable(int dim, int rank);
// shapes whose gauge and slices the persistent block builds, and the doubles
// of per-wavefront scratch that needs
bool bp_persistent_regauge_supported(int dim, int rank);
int bp_persistent_regauge_table(int dim, int rank);
int bp_persistent_sites_per_tile(int dim, int rank);
hipError_t launch_regauge(const DeviceBatch &b, hipStream_t s);
// shapes the register-path regauge handles (all legs of dimension dim)
bool regauge_reg_supported(int dim, int rank);
// tensor buffers of the per-site regauge of r: one when every gauged leg has
// dimension <= 6 (fiber-wise products in place), else two
__host__ __device__ inline int regauge_site_buffers(const SiteRec &r) {
    for (int l = 0; l < r.rank; ++l)
        if (!((r.open_mask >> l) & 1) && r.dim[l] > 6) return 2;
    return 1;
}
// dynamic LDS (doubles) of the per-site regauge of r: its tensor buffers and
// a d x d transform per gauged slot
inline size_t regauge_site_lds_doubles(const SiteRec &r) {
    size_t n = (size_t)regauge_site_buffers(r) * (size_t)r.size;
    for (int l = 0; l < r.rank; ++l)
        if (!((r.open_mask >> l) & 1)) n += (size_t)r.dim[l] * (size_t)r.dim[l];
    return n;
}
// shapes of the one-site register regauge (k_regauge_wide), and its sites per tile
bool regauge_wide_supported(int dim, int rank);
int regauge_wide_sites(int dim, int rank);
// doubles of the per-wavefront LDS transform table of a register regauge tile
int regauge_table_doubles(int dim, int rank);
hipError_t launch_clusters(const DeviceBatch &b, hipStream_t s);
hipError_t launch_combine(const DeviceBatch &b, hipStream_t s);

}  // namespace pne

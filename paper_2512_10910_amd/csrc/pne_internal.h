// Internal types shared by the host runtime and the gfx950 kernels.
#pragma once

#include <cstdint>

namespace pne {

constexpr int kMaxRank = 8;    // leg slots per site
constexpr int kMaxDim = 16;    // largest leg dimension
constexpr int kMaxLab = 8;     // index labels touched by one contraction step
constexpr int kMaxVerts = 16;  // sites in one cluster
constexpr int kMaxOpenOut = 64;  // entries of an open-index output tensor
constexpr int kMaxParts = 32;    // user partitions of one network

// One site of one network in a batch (device table).
struct SiteRec {
    const double *t;      // input tensor, FP64, C order over slots
    int64_t slice_off;    // element offset of the regauged slices in the slice arena
    int32_t msg_off;      // offset of the site's incoming messages (slot-major)
    int32_t vside_mask;   // bit l set when this site is the second site of slot l's bond
    int32_t rank;
    int32_t size;         // product of dims
    int32_t net;          // network index in the batch
    int32_t open_mask;    // bit l set when slot l is an open leg
    int32_t vac_off;      // open sites: offset in the FP64 vacuum buffer, else -1
    int32_t pad;
    int32_t dim[kMaxRank];
    int32_t stride[kMaxRank];
    int32_t moff[kMaxRank];  // offset of slot l's incoming message relative to msg_off
    int32_t dst[kMaxRank];   // absolute offset of the incoming message that slot l's
                             // outgoing message becomes (partner slot, or itself if open)
};

// A BP tile: sites of one network sharing rank and leg dims.
struct BpTile {
    int32_t site_begin;   // index into the tile-site list
    int32_t n_sites;
    int32_t net;
    int32_t rank;
    int32_t size;         // tensor entries per site
    int32_t n_os;         // outputs (sum of dims) per site
    int32_t first;        // 1 for the network's first tile (writes its bookkeeping)
    int32_t dc;           // common leg dimension (2..6) for specialised code, else 0
    int32_t reg;          // 1: register path (all legs of dimension dc)
    int32_t pad;
};

// A network run by the persistent per-network BP kernel.
struct FusedNet {
    int32_t net;          // network index in the batch
    int32_t msg_base;     // absolute offset of the network's first message
    int32_t msg_size;     // doubles of messages
    int32_t site_base;    // global index of the network's first site
    int32_t n_sites;
    int32_t group_begin;  // shape groups of the network
    int32_t n_groups;
    int32_t list_begin;   // site list (local site ids, group after group)
    int32_t scratch;      // doubles of per-wavefront scratch
    int32_t colors;       // 2: bipartite, red-black schedule in one buffer; 1: Jacobi, two buffers
    int32_t rg_inline;    // 1: the block also builds the gauge and slices of every site
    int32_t cl_fused;     // 1: ... and contracts its clusters and sums its terms (closed network)
    int32_t class_begin;  // the network's plan classes (cl_fused)
    int32_t n_classes;
    int32_t prio;         // wave issue priority (0..3): higher for networks with more work per step
    int64_t w_base;       // the network's first cluster weight (cl_fused)
};

// Sites of one network with all legs of dimension dc and rank `rank`.
struct FusedGroup {
    int32_t dc, rank;
    int32_t spw;          // sites per tile
    int32_t list_off;     // first entry in the network's site list
    int32_t n_sites;
    int32_t nt;           // tiles per wavefront step
    int32_t color;        // site colour (0/1) under the red-black schedule, else 0
    int32_t pad;
};

// Per-network BP state.  Sweep k reads message buffer k&1, writes buffer
// (k+1)&1 and folds its residual into res_acc[k%3]; a network stopped at
// sweep s keeps its final messages in buffer (s+1)&1.
struct NetState {
    int32_t stop;       // sweep at which BP stopped, -1 while running
    int32_t iters;      // sweeps performed (stop + 1)
    int32_t parity;     // buffer holding the final messages
    int32_t status;     // 0 ok, else a negative pne_status
    unsigned long long res_acc[3];  // per-sweep residual maxima (bits of doubles >= 0)
    // smallest residual so far and the sweep that reached it, double-buffered
    // for the per-launch sweeps: the test of sweep k reads slot k&1 and its
    // first tile writes the update with sweep k-1's residual to the other slot
    double best[2];
    int32_t best_at[2];
    double residual;    // residual of the last sweep
    double log_bp;
    int32_t sign_bp;
    int32_t converged;
    // persistent block phase timestamps (device wall clock ticks): start,
    // end of BP, end of the in-block gauge + slices
    unsigned long long t_start, t_bp, t_rg;
};

// A contraction step of a cluster plan: absorb one site's slice into the
// running frontier tensor F.  Output labels come first in F_next's C order.
struct StepDesc {
    int32_t vert;        // position of the absorbed site in the instance record
    int32_t n_out;       // entries of F_next
    int32_t n_sum;       // entries of the summed (shared) index space
    int32_t n_ol;        // output labels
    int32_t n_sl;        // summed labels
    int32_t n_xl;        // legs of the absorbed slice
    int32_t out_dim[kMaxLab];
    int32_t out_fs[kMaxLab];   // stride in F of each output label (0 if new)
    int32_t out_xl[kMaxLab];   // slice leg of each output label (-1 if from F)
    int32_t sum_dim[kMaxLab];
    int32_t sum_fs[kMaxLab];
    int32_t sum_xl[kMaxLab];
    int32_t x_excited[kMaxLab];  // 1 when the slice leg is an excited bond leg
    int32_t ent;         // first StepEnt of the step (n_out output entries, then n_sum
                         // summed entries), or -1 when the class has no entry tables
};

// Precomputed index of one output entry or one summed entry of a step, in
// the order the contraction visits them (last label fastest): f is its
// offset in F (for an output entry, F's part of it), xdig the slice index
// digit of each slice leg m in bits 4m..4m+3.  An instance's slice offset is
// the sum of digit x stride over its slice legs.
struct StepEnt {
    int32_t f;
    uint32_t xdig;
};

// A class of clusters with the same contraction plan.
struct ClassDesc {
    // device tables of the class, kept by the context once per plan (null in
    // the plan's own copy)
    const struct InstStep *tab;  // InstStep records, instance-major (n_steps, or n_verts for a cycle, each)
    const int32_t *iw;           // weight offset of each instance from its network's weight base
    int32_t step_begin;  // index into the step table
    int32_t n_steps;
    int32_t n_verts;
    int32_t max_f;       // largest frontier (entries)
    int32_t group;       // lanes per instance (power of two, <= 64)
    int32_t out_size;    // entries of the result tensor (1 for closed clusters)
    // filled per batch
    int32_t n_inst;      // instances per network
    int32_t pnet_begin;  // first PlanNet of the networks sharing the class's plan
    int32_t n_pnets;
    int32_t scalar;      // 1: frontier of one entry throughout (every leg of dimension 1)
    int32_t loop_e;      // > 0: a simple cycle of legs of dimension loop_e, evaluated as the
                         // trace of a matrix product (records in cycle order)
    int32_t max_sum;     // > 0: every step has StepEnt tables; the largest summed space
};

// One step of one instance: where the absorbed slice's block starts (element
// offset from the network's slice base, excited legs already at index 1)
// and the strides of the slice legs the step uses.  For a cycle class the
// records follow the cycle, xs[0] being the leg towards the previous site
// and xs[1] the leg towards the next.
struct InstStep {
    int32_t xoff;
    int32_t xs[kMaxLab];
    int32_t pad[3];
};

// A network in the batch that uses a given plan.
struct PlanNet {
    int64_t slice_base;  // element offset of the network's first slice
    int64_t w_base;      // offset of the network's first cluster weight
    int32_t net;         // the network's index in the batch
    int32_t pad;
};

// A block of cluster work: `count` consecutive instances of one class.
struct ClusterBlock {
    int32_t cls;
    int32_t flat_begin;  // first (network, instance) pair, network-major: net * n_inst + instance
    int32_t count;
    int32_t pad;
};

// Per-network combine description (geometry tables are shared).
struct CombineRec {
    int64_t w_base;        // start of the network's weights in the weight buffer
    int32_t n_clusters;
    int32_t pad0;
    int32_t geo;           // geometry table index
    int32_t site_begin;    // first global site of the network
    int32_t n_sites;
    int32_t vac_a, vac_b;  // vacuum offsets of the open sites (-1 if none)
    int32_t pa, pb;        // open dims of A and B (1 if absent)
    int32_t open_off;      // first entry of the network's pa*pb open output (-1: closed network)
    int32_t cumulant;      // 1: closed network summed in exponentiated (cumulant) form
};

// Per-network device result.
struct NetResult {
    double log_abs;
    double log_bp;
    double sum;            // closed networks: the retained-term sum S (Z = Z_BP (1+S))
    double dangling;       // largest excited norm of a single-leg slice (0 at a BP fixed point)
    double err_est;        // first-order estimate of the term precision's error (see pne_result)
    int32_t sign;
    int32_t status;
};  // an open network's output tensor goes to the batch's open-output buffer

// Geometry-level combine tables.
struct GeoRec {
    int32_t K;
    int32_t n_buckets;     // buckets of (type, size), contiguous cluster ranges
    int32_t bucket_begin;  // index into the bucket table
    int32_t pair_begin;    // index into the overlap-pair tables
    int32_t n_pairs;
    int32_t pair_cat_begin;  // categories of pairs (contiguous ranges)
    int32_t n_pair_cats;
    int32_t listed;        // 1: the configurations are listed (user partitions)
    int32_t coll_begin;    // listed: index of the first offset in the collection offsets
    int32_t n_colls;       // listed: number of retained configurations
    int32_t coll_cl_begin; // listed: index of the first entry in the collection clusters
    int32_t coef_begin;    // listed with sub-partitions: first coefficient; -1: every coefficient is 1
};

struct Bucket {
    int32_t type;    // 0 closed, 1 touches A only, 2 touches B only, 3 touches both
    int32_t size;    // cluster size (bonds)
    int32_t begin;   // cluster range [begin, end) within the network
    int32_t end;
    int32_t w_begin; // weight offset of the first cluster (weights are contiguous)
    int32_t osz;     // weight entries per cluster
};

struct PairCat {
    int32_t t1, t2;  // types of the two clusters (t1 >= t2 after ordering)
    int32_t begin, end;  // range in the pair table
};

}  // namespace pne

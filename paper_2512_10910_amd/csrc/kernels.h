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
    const BpTile *tiles = nullptr;
    int n_tiles = 0;
    const int *tile_sites = nullptr;
    size_t bp_lds = 0;             // dynamic LDS of the sweep kernel
    const BondRec *bonds = nullptr;
    int n_bonds = 0;
    NetState *state = nullptr;
    int n_nets = 0;
    int *n_active = nullptr;
    // buffers
    double *msg0 = nullptr, *msg1 = nullptr;
    double *xg = nullptr;
    void *slices = nullptr;
    int precision = 0;
    double *site_log = nullptr;
    int *site_sign = nullptr;
    double *vac = nullptr;
    size_t regauge_lds = 0;
    // clusters
    const ClassDesc *classes = nullptr;
    const StepDesc *steps = nullptr;
    const ClusterBlock *cblocks = nullptr;
    int n_cblocks = 0;
    const int *inst_site = nullptr;       // global site ids, n_verts per instance
    const uint32_t *inst_slots = nullptr;
    const int64_t *inst_wout = nullptr;   // per instance: weight offset
    const int64_t *inst_rec = nullptr;    // per instance: offset into inst_site/inst_slots
    size_t cluster_lds = 0;
    double *w = nullptr;
    // combine
    const CombineRec *crec = nullptr;
    const GeoRec *geos = nullptr;
    const Bucket *buckets = nullptr;
    const int *pair_a = nullptr, *pair_b = nullptr;
    const PairCat *pair_cats = nullptr;
    NetResult *results = nullptr;
};

// kernel identifiers for per-kernel timing
enum KernelId { KID_INIT = 0, KID_SWEEP, KID_FINISH, KID_GAUGE, KID_REGAUGE, KID_CLUSTERS, KID_COMBINE, KID_COUNT };

hipError_t launch_init(const DeviceBatch &b, hipStream_t s);
hipError_t launch_sweep(const DeviceBatch &b, hipStream_t s);
hipError_t launch_finish(const DeviceBatch &b, double tol, int max_iter, hipStream_t s);
hipError_t launch_gauge(const DeviceBatch &b, hipStream_t s);
hipError_t launch_regauge(const DeviceBatch &b, hipStream_t s);
hipError_t launch_clusters(const DeviceBatch &b, hipStream_t s);
hipError_t launch_combine(const DeviceBatch &b, hipStream_t s);

}  // namespace pne

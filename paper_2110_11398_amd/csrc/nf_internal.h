// Internal declarations shared by the HIP translation units of libabacus_nf.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/abacus_nf.h"

namespace anf {

// One periodic box, resident on the device for the binning and the work list.
struct BoxDev {
    int64_t offset;     // first particle of the box in the input array
    int64_t n;          // particles in the box
    double L;           // side
    double s;           // K / L, computed once on the host in FP64
    int32_t K;          // cells per side
    int32_t cell_base;  // global index of the box's first cell
};

// Per-box constants of one forces call, in cell-width units.
struct ForceBox {
    float c0, c1, c2;   // spline: g = min(rinv^3, c0 + r2 * (c1 * rinv + c2))
    float eps2;         // Plummer: g = (r2 + eps2)^(-3/2)
    double scale;       // G*m / w^2: converts a cell-unit sum into an acceleration
    float scalef;       // the same in FP32 (plain FP32 mode)
    float kde_ib2;      // density: weight = max(0, kde_c - r2 * kde_ib2), kde_ib2 = 1/b^2 (cell units)
    float kde_c;        // 1 + (offset added to r2 in the pair chain) * kde_ib2
    int32_t pad;
};

// One unit of work of the persistent force kernel: a tile of sinks of one
// cell against one part of that cell's near-field source list.
struct Item {
    int32_t cell, tile, part, box;
};

constexpr int kNumClasses = 64;
// The persistent kernel drains the item list through kQueues queues: the list
// is cut into blocks of kQueueBlock consecutive items (spatially close cells of
// one cost class), block b belongs to queue b % kQueues, and a workgroup starts
// on queue blockIdx % kQueues -- the compute die (XCD) the hardware dispatches
// it to -- and steals from the other queues once its own is empty.  Neighbouring
// cells then share one XCD's L2.
constexpr int kQueues = 8;
constexpr int kQueueBlock = 32;
// Items of the light cost classes (an item of class >= kLightClass costs under ~1024 source iterations x sinks
// per lane) are claimed kLightClaim queue slots per atomic: sparse regions hold millions of such items, and one
// atomic per item on the queue cursors would bound the kernel.
constexpr int kLightClass = 44;
constexpr int kLightClaim = 8;

// Device-side state of the work list of one forces call.
struct WorkState {
    unsigned long long interactions;  // sum over cells of n_c * sources(c)
    unsigned long long part_demand;   // partial slots needed at the base part size
    int32_t n_items;                  // items emitted (clamped to the capacity)
    int32_t cursor[kQueues];          // next item of each queue of the persistent kernel
    int32_t part_iters;               // effective part length (source iterations per lane)
    int32_t overflow;                 // non-zero when a list outgrew its capacity
    unsigned long long base_items;    // items with every source list unsplit
    unsigned long long split_items;   // items of cells whose source list is split
    int32_t class_count[kNumClasses];
    int32_t class_fill[kNumClasses];
    int32_t class_base[kNumClasses];
    int32_t light_slot[kQueues];       // first slot of each queue that holds a light item
};

// Sink tiles of one cell.  The n sinks form g = ceil(n / S) groups of S (one
// group per lane); a tile of G groups gives each group L = 64 / G lanes (at most
// max_lanes), which split the sources between them.  Whole tiles of 64 groups
// (L = 1) come first.  A rest of r < 64 groups is one tile when that tile keeps
// at least 7/8 of the wave's lanes busy, when r is a power of two, or when the
// cut below would need more than max_lanes lanes per group; otherwise a tile of
// the largest power of two k < r groups (L = 64 / k, every lane busy) is cut
// off and the rest follows the same rule.
// So every tile but a cell's last fills its wave (e.g. 43 groups: 32 with L = 2,
// 8 with L = 8, 3 with L = 21), and tile 0 has the fewest lanes per group.
struct TileGeom {
    int L, G;     // lanes per group, groups (capacity G * S sinks)
    int t0, nt;   // first sink of the tile within the cell, sinks in the tile
};

// One tile of a rest of r groups: returns true when it takes the whole rest.
__host__ __device__ inline bool rest_tile(int r, int max_lanes, int &L, int &G) {
    int L0 = 64 / r;
    if (L0 > max_lanes) L0 = max_lanes;
    const int k = 1 << (31 - __builtin_clz((unsigned)r));   // largest power of two <= r
    if (k == r || 8 * r * L0 >= 7 * 64 || 64 / k > max_lanes) {
        L = L0;
        G = 64 / L0;
        return true;
    }
    L = 64 / k;
    G = k;
    return false;
}

__host__ __device__ inline int tile_count(int n, int S, int max_lanes) {
    if (n <= 0) return 0;
    const int g = (n + S - 1) / S;
    int count = g / 64, r = g - 64 * (g / 64);
    while (r > 0) {
        int L, G;
        count++;
        if (rest_tile(r, max_lanes, L, G)) break;
        r -= G;
    }
    return count;
}

// Tile number `tile` (0 <= tile < tile_count) of a cell with n > 0 sinks.
__host__ __device__ inline TileGeom tile_at(int n, int S, int max_lanes, int tile) {
    TileGeom t;
    const int g = (n + S - 1) / S;
    const int full = g / 64;
    if (tile < full) {
        t.L = 1;
        t.G = 64;
        t.t0 = tile * 64 * S;
        t.nt = n - t.t0 < 64 * S ? n - t.t0 : 64 * S;
        return t;
    }
    int r = g - 64 * full, t0 = full * 64 * S;
    if (r <= 0) {   // no such tile: an empty one
        t.L = 1;
        t.G = 64;
        t.t0 = n;
        t.nt = 0;
        return t;
    }
    for (int k = full;; k++) {
        int L, G;
        const bool last = rest_tile(r, max_lanes, L, G);
        if (k == tile || last) {
            t.L = L;
            t.G = G;
            t.t0 = t0;
            t.nt = last ? n - t0 : G * S;
            return t;
        }
        t0 += G * S;
        r -= G;
    }
}

// Box of particle i: the last box whose offset is <= i (boxes partition the input in order).
__device__ inline int box_of_particle(const BoxDev *boxes, int n_boxes, int64_t i) {
    int lo = 0, hi = n_boxes - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (boxes[mid].offset <= i) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Box of global cell c: the last box whose cell_base is <= c.
__device__ inline int box_of_cell(const BoxDev *boxes, int n_boxes, int32_t c) {
    int lo = 0, hi = n_boxes - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (boxes[mid].cell_base <= c) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// (The definitions above are all the force kernel takes from this header.)

// Error reporting: the first device error since the last abacus_nf_sync.
int *device_error_word(int device);   // host accessor (allocates on first use)

// Launch helpers (cells.hip)
hipError_t launch_set_boxes(const abacus_nf_box *boxes, int n_boxes, const int32_t *cell_base,
                            BoxDev *dst, hipStream_t st);
hipError_t launch_bin(const float *pos, int64_t n, const BoxDev *boxes, int n_boxes, int32_t *keys,
                      int32_t *vals, int *err, hipStream_t st);
size_t radix_temp_bytes(int64_t n);
hipError_t radix_sort_pairs(int32_t *keys, int32_t *vals, int32_t *keys_tmp, int32_t *vals_tmp,
                            void *temp, int64_t n, int key_bits, hipStream_t st, int32_t **keys_out,
                            int32_t **vals_out);
size_t scan_temp_bytes(int64_t n);
hipError_t scan_i32_max_inclusive(const int32_t *in, int32_t *out, int64_t n, void *temp, hipStream_t st);
hipError_t scan_i64_add_exclusive(const int64_t *in, int64_t *out, int64_t n, void *temp, hipStream_t st);
hipError_t launch_cell_start(const int32_t *keys_sorted, int64_t n, int64_t n_cells, int32_t *endpos,
                             int32_t *cell_start, void *scan_temp, hipStream_t st);
hipError_t launch_gather(const float *pos, const int32_t *perm, const int32_t *keys_sorted, int64_t n,
                         const BoxDev *boxes, int n_boxes, float4 *spos, hipStream_t st);
hipError_t launch_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t st);

// Cell multipoles (multipoles.hip)
int multipole_components(int p);
int multipole_max_order();
size_t multipole_partial_doubles(int64_t n_total, int p);   // unit partials buffer size
hipError_t launch_multipoles(const float4 *spos, const int32_t *keys, const int32_t *cs, const BoxDev *boxes,
                             int n_boxes, int64_t n,
                             int64_t n_cells, int p, const double *mass_host, double *mass_dev, double *partials,
                             double *out, int device, hipStream_t st);

// Far field from cell Taylor series (taylor.hip)
int taylor_max_order();
hipError_t launch_taylor(const float4 *spos, const int32_t *keys, const int32_t *perm, const BoxDev *boxes,
                         int n_boxes, int64_t n, int64_t n_cells, int p, const double *taylor, float *acc,
                         int device, hipStream_t st);

// Work list and forces (forces.hip)
struct ForcesArgs {
    const float4 *spos;
    const int32_t *cell_start;
    const int32_t *perm;
    const int32_t *keys;
    const BoxDev *boxes;
    const ForceBox *fbox;
    int n_boxes;
    int64_t n_total;
    int64_t n_cells;
    int R;
    Item *items;
    int64_t item_capacity;
    WorkState *ws;
    int32_t *cell_nsrc;
    int32_t *cell_parts;
    int64_t *cell_pdem;
    int64_t *cell_pbase;
    double *partials;
    int64_t partial_capacity;
    float *acc;
    double *acc64;   // FP64 accelerations instead of acc (nullptr: FP32 output)
    float *rho;      // density output (nullptr: forces only)
    unsigned long long *amax;   // [n_cells] bits of the largest |a|^2 written in each cell (FP64)
    int *err;
    abacus_nf_kind kind;
    abacus_nf_sum mode;
    abacus_nf_tuning tune;
    int grid;        // persistent-kernel workgroups
    void *scan_temp;
};

hipError_t launch_set_force_boxes(const double *eps, const double *gm, const double *kde_b, abacus_nf_kind kind,
                                  const abacus_nf_box *boxes, int n_boxes, ForceBox *dst, hipStream_t st);
hipError_t build_work_list(const ForcesArgs &a, hipStream_t st);
hipError_t launch_forces(const ForcesArgs &a, hipStream_t st);
hipError_t launch_finalize(const ForcesArgs &a, hipStream_t st);
int forces_grid(const abacus_nf_tuning &t, abacus_nf_kind kind, abacus_nf_sum mode, bool kde, int device);
hipError_t launch_count_interactions(const ForcesArgs &a, hipStream_t st);

// Leapfrog time stepping (kdk.hip)
hipError_t upload_box_doubles(const double *host, int n_boxes, double *dev, hipStream_t st);
hipError_t launch_kick(float *vel, const float *acc, int64_t n, const BoxDev *boxes, int n_boxes, const double *dt,
                       int device, hipStream_t st);
hipError_t launch_drift(float *pos, const float *vel, int64_t n, const BoxDev *boxes, int n_boxes, const double *dt,
                        int device, hipStream_t st);
hipError_t launch_reorder(float *const *vec3, int n_vec3, int64_t *ids, int32_t *perm, int64_t n, void *scratch,
                          int device, hipStream_t st);
size_t timestep_partial_doubles(int64_t n);
hipError_t launch_timestep(const float *vel, const float *acc, const unsigned long long *amax, const int32_t *keys,
                           const int32_t *perm, const int32_t *cs, const BoxDev *boxes, int n_boxes, int64_t n,
                           double *partials, unsigned long long *dmin, hipStream_t st);
hipError_t launch_fill_u64(unsigned long long *p, int64_t n, unsigned long long v, hipStream_t st);
// Words of the per-box minima buffer of the timestep criterion (slots per box, then one final word per
// box), and where the final words start.
size_t timestep_min_words(int n_boxes);
size_t timestep_min_offset(int n_boxes);

// The step-size criterion of a handle with buffers the caller provides (api.hip): partials of at least
// timestep_partial_doubles(n_total) doubles and per-box minima of at least timestep_min_words(n_boxes)
// words.  The argument checks of abacus_nf_timestep come first; EINVAL when a buffer is missing or too small.
int timestep_with_buffers(abacus_nf_cells h, const float *vel, const float *acc, double eta, double *dt_out,
                          double *partials, size_t partial_doubles, unsigned long long *dmin, size_t dmin_words,
                          void *hip_stream);
int handle_boxes(abacus_nf_cells h);   // boxes of a handle (0 for NULL)
// The argument and state checks of abacus_nf_timestep alone (no HIP call).
int timestep_arguments(abacus_nf_cells h, const float *vel, const float *acc, double eta, double *dt_out);

}  // namespace anf

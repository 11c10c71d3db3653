// Near-field force: device work list and the persistent pairwise kernel.
//
// The operation is the direct sum of Sec. 3.1 (near field = cells within R,
// explicit periodic images) with the spline or Plummer softening of Sec. 2.5
// and Sec. 5.2.  The paper runs it as CUDA kernels on host-packaged work units
// ("Index Near Force Pencils", "spatially compact GPU work units", Sec. 4.3 and
// Sec. 4.5).  Here the work list is built on the device and one persistent
// launch drains it:
//
//   k_wl_cells    per cell: occupancy n_c, near-field source count, pair total
//   k_wl_plan     scales the source-part length so partial slots fit
//   k_wl_count    per cell: tiles x parts, cost class (histogram over classes)
//   k_wl_classes  class offsets (heaviest items first), capacity checks
//   k_wl_emit     items written in class order
//   k_forces      persistent waves pop items: sink tile in VGPRs, sources staged
//                 through the wave's LDS region with the periodic cell offset
//                 applied, FP32 pair math, FP32 / two-sum / FP64 accumulation,
//                 ordered cross-lane reduction, output in input order
//   k_finalize    sums the parts of sinks whose source list was split (FP64)
//
// Numbers are in cell-width units: positions are relative to the sink cell's
// centre, so the pair terms need no large-coordinate cancellation.
#include <climits>
#include <cstring>
#include <cmath>

#include "nf_internal.h"

namespace anf {

namespace {

constexpr int kWaves = 4;                 // independent waves per workgroup
constexpr int kThreads = 64 * kWaves;
constexpr float kTiny = 1e-20f;           // keeps rsqrt finite for coincident pairs
constexpr float kFar = 1e18f;             // padding source: its terms underflow to exactly 0

inline unsigned grid_for(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

// ---------------------------------------------------------------- per-box constants

constexpr int kFBoxChunk = 48;
struct FBoxChunk {
    ForceBox f[kFBoxChunk];
    int first, count;
};

__global__ void k_set_fbox(FBoxChunk c, ForceBox *dst) {
    int i = threadIdx.x;
    if (i < c.count) dst[c.first + i] = c.f[i];
}

// ---------------------------------------------------------------- near-field columns

// The near field of cell (cx, cy, cz) is (2R+1)^2 columns of neighbouring
// cells, each a run of 2R+1 consecutive cells along z.  In the sorted layout
// a run is a contiguous slot range, split in two where it wraps through the
// periodic z boundary.  czref turns the stored z cell index of a source into
// its offset from the sink cell: dz = cz_src - czref.
struct ColSeg {
    int32_t src0, len0, src1, len1;
    float czref0, czref1;
};

__device__ inline void column_segments(const int32_t *__restrict__ cs, int colbase, int cz, int K, int R,
                                       ColSeg &o) {
    const int z0 = cz - R, z1 = cz + R;
    if (z0 < 0) {            // images below the box first, then the cells from 0
        o.src0 = cs[colbase + z0 + K];
        o.len0 = cs[colbase + K] - o.src0;
        o.czref0 = (float)(cz + K);
        o.src1 = cs[colbase];
        o.len1 = cs[colbase + z1 + 1] - o.src1;
        o.czref1 = (float)cz;
    } else if (z1 >= K) {    // cells up to K-1, then images above the box
        o.src0 = cs[colbase + z0];
        o.len0 = cs[colbase + K] - o.src0;
        o.czref0 = (float)cz;
        o.src1 = cs[colbase];
        o.len1 = cs[colbase + z1 - K + 1] - o.src1;
        o.czref1 = (float)(cz - K);
    } else {
        o.src0 = cs[colbase + z0];
        o.len0 = cs[colbase + z1 + 1] - o.src0;
        o.czref0 = (float)cz;
        o.src1 = 0;
        o.len1 = 0;
        o.czref1 = 0.f;
    }
}

__device__ inline int wrap(int v, int K) { return v < 0 ? v + K : (v >= K ? v - K : v); }

// Number of near-field sources of cell c.
__device__ inline int cell_sources(const int32_t *__restrict__ cs, const BoxDev &B, int lin, int R) {
    const int K = B.K;
    const int cz = lin % K, cy = (lin / K) % K, cx = lin / (K * K);
    int total = 0;
    for (int dx = -R; dx <= R; dx++) {
        const int ex = wrap(cx + dx, K);
        for (int dy = -R; dy <= R; dy++) {
            const int ey = wrap(cy + dy, K);
            ColSeg o;
            column_segments(cs, B.cell_base + (ex * K + ey) * K, cz, K, R, o);
            total += o.len0 + o.len1;
        }
    }
    return total;
}

// Tiles, parts and cost class of one cell.
struct CellPlan {
    int tiles, parts, cls;
    int64_t items;
};

__device__ inline CellPlan plan_cell(int n, int nsrc, int S, int max_lanes, int part_iters) {
    CellPlan p;
    if (n <= 0) {
        p.tiles = p.parts = 0;
        p.items = 0;
        p.cls = kNumClasses - 1;
        return p;
    }
    p.tiles = tile_count(n, S, max_lanes);
    const int L0 = tile_at(n, S, max_lanes, 0).L;               // the heaviest tile: fewest lanes per group
    const int64_t iters = ((int64_t)nsrc + L0 - 1) / L0;        // source iterations per lane
    int64_t parts = (iters + part_iters - 1) / part_iters;
    if (parts < 1) parts = 1;
    if (parts > nsrc) parts = nsrc > 0 ? nsrc : 1;
    p.parts = (int)parts;
    p.items = (int64_t)p.tiles * p.parts;
    // cost of one item ~ iterations per lane x sinks per lane; classes are half octaves, heaviest first
    const double cost = (double)(iters / parts + 1) * S + 16.0;
    int cls = kNumClasses - 1 - (int)(2.0 * log2(cost));
    p.cls = cls < 0 ? 0 : (cls >= kNumClasses ? kNumClasses - 1 : cls);
    return p;
}

// ---------------------------------------------------------------- work-list kernels

__global__ void k_wl_clear(WorkState *ws, int part_iters) {
    int t = threadIdx.x;
    if (t == 0) {
        ws->interactions = 0;
        ws->part_demand = 0;
        ws->base_items = 0;
        ws->split_items = 0;
        ws->n_items = 0;
        for (int q = 0; q < kQueues; q++) ws->cursor[q] = 0;
        ws->part_iters = part_iters;
        ws->overflow = 0;
    }
    if (t < kNumClasses) {
        ws->class_count[t] = 0;
        ws->class_fill[t] = 0;
        ws->class_base[t] = 0;
    }
}

__device__ inline unsigned long long wave_sum_u64(unsigned long long v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// Per cell: source count, exact pair total, and the demand of the base part length.
__global__ __launch_bounds__(256) void k_wl_cells(const int32_t *__restrict__ cs, const BoxDev *__restrict__ boxes,
                                                  int n_boxes, int64_t n_cells, int R, int S, int max_lanes,
                                                  int32_t *__restrict__ cell_nsrc, WorkState *ws) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long inter = 0, pdem = 0, base_items = 0, split_items = 0;
    if (c < n_cells) {
        const int n = cs[c + 1] - cs[c];
        int nsrc = 0;
        if (n > 0) {
            const int b = n_boxes > 1 ? box_of_cell(boxes, n_boxes, (int32_t)c) : 0;
            const BoxDev B = boxes[b];
            nsrc = cell_sources(cs, B, (int)(c - B.cell_base), R);
            inter = (unsigned long long)n * (unsigned long long)nsrc;
            const CellPlan p = plan_cell(n, nsrc, S, max_lanes, ws->part_iters);
            base_items = (unsigned long long)p.tiles;
            if (p.parts > 1) {
                pdem = (unsigned long long)p.parts * (unsigned long long)n;
                split_items = (unsigned long long)p.items;
            }
        }
        cell_nsrc[c] = nsrc;
    }
    inter = wave_sum_u64(inter);
    pdem = wave_sum_u64(pdem);
    base_items = wave_sum_u64(base_items);
    split_items = wave_sum_u64(split_items);
    if ((threadIdx.x & 63) == 0) {
        if (inter) atomicAdd(&ws->interactions, inter);
        if (pdem) atomicAdd(&ws->part_demand, pdem);
        if (base_items) atomicAdd(&ws->base_items, base_items);
        if (split_items) atomicAdd(&ws->split_items, split_items);
    }
}

// Lengthen the source parts until the partial slots and the items fit.
__global__ void k_wl_plan(WorkState *ws, int64_t partial_capacity, int64_t item_capacity, int64_t n_total) {
    if (threadIdx.x != 0) return;
    const int64_t pbudget = partial_capacity - n_total;
    const int64_t ibudget = item_capacity - (int64_t)ws->base_items;
    int64_t f = 1;
    const int64_t pd = (int64_t)ws->part_demand, id = (int64_t)ws->split_items;
    if (pd > 0) {
        int64_t fp = pbudget > 0 ? (pd + pbudget - 1) / pbudget : INT_MAX;
        if (fp > f) f = fp;
    }
    if (id > 0) {
        int64_t fi = ibudget > 0 ? (id + ibudget - 1) / ibudget : INT_MAX;
        if (fi > f) f = fi;
    }
    int64_t it = (int64_t)ws->part_iters * f;
    ws->part_iters = (int32_t)(it > INT_MAX ? INT_MAX : it);
}

__global__ __launch_bounds__(256) void k_wl_count(const int32_t *__restrict__ cs, const int32_t *__restrict__ cell_nsrc,
                                                  int64_t n_cells, int S, int max_lanes, WorkState *ws,
                                                  int32_t *__restrict__ cell_parts, int64_t *__restrict__ cell_pdem) {
    __shared__ int32_t hist[kNumClasses];
    if (threadIdx.x < kNumClasses) hist[threadIdx.x] = 0;
    __syncthreads();
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int part_iters = ws->part_iters;
    if (c < n_cells) {
        const int n = cs[c + 1] - cs[c];
        const CellPlan p = plan_cell(n, cell_nsrc[c], S, max_lanes, part_iters);
        cell_parts[c] = p.parts;
        cell_pdem[c] = p.parts > 1 ? (int64_t)p.parts * n : 0;
        if (p.items > 0) atomicAdd(&hist[p.cls], (int32_t)p.items);
    }
    __syncthreads();
    if (threadIdx.x < kNumClasses && hist[threadIdx.x]) atomicAdd(&ws->class_count[threadIdx.x], hist[threadIdx.x]);
}

__global__ void k_wl_classes(WorkState *ws, int64_t item_capacity, const int64_t *__restrict__ pbase,
                             const int64_t *__restrict__ pdem, int64_t n_cells, int64_t partial_capacity,
                             int *err) {
    if (threadIdx.x != 0) return;
    int64_t run = 0;
    for (int k = 0; k < kNumClasses; k++) {
        ws->class_base[k] = (int32_t)(run < INT_MAX ? run : INT_MAX);
        ws->class_fill[k] = 0;
        run += ws->class_count[k];
    }
    int64_t need_p = n_cells > 0 ? pbase[n_cells - 1] + pdem[n_cells - 1] : 0;
    bool over = run > item_capacity || need_p > partial_capacity;
    // on overflow nothing is emitted and nothing is computed: the error is
    // reported by abacus_nf_sync and the output is left unwritten
    ws->n_items = over ? 0 : (int32_t)run;
    for (int q = 0; q < kQueues; q++) ws->cursor[q] = 0;
    // slot j of queue x holds item ((j / kQueueBlock) * kQueues + x) * kQueueBlock + j % kQueueBlock, increasing
    // in j: the first slot of each queue at or past the first light item
    const int64_t L0 = ws->class_base[kLightClass];
    const int64_t B = L0 / kQueueBlock, o = L0 % kQueueBlock;
    for (int x = 0; x < kQueues; x++) {
        const int64_t bq = B > x ? (B - x + kQueues - 1) / kQueues : 0;   // first block of queue x at or past B
        const int64_t slot = bq * kQueueBlock + (bq * kQueues + x == B ? o : 0);
        ws->light_slot[x] = (int32_t)(slot < INT_MAX ? slot : INT_MAX);
    }
    ws->overflow = over ? 1 : 0;
    if (over) atomicCAS(err, 0, ABACUS_NF_ECAPACITY);
}

__global__ __launch_bounds__(256) void k_wl_emit(const int32_t *__restrict__ cs, const int32_t *__restrict__ cell_nsrc,
                                                 const int32_t *__restrict__ cell_parts,
                                                 const BoxDev *__restrict__ boxes, int n_boxes, int64_t n_cells,
                                                 int S, int max_lanes, WorkState *ws, Item *__restrict__ items,
                                                 int64_t item_capacity) {
    __shared__ int32_t cnt[kNumClasses];
    __shared__ int32_t bbase[kNumClasses];
    if (threadIdx.x < kNumClasses) cnt[threadIdx.x] = 0;
    __syncthreads();
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    CellPlan p;
    p.items = 0;
    p.cls = 0;
    p.tiles = p.parts = 0;
    int local = 0;
    if (c < n_cells) {
        const int n = cs[c + 1] - cs[c];
        if (n > 0) {
            p = plan_cell(n, cell_nsrc[c], S, max_lanes, ws->part_iters);
            p.parts = cell_parts[c];
            p.items = (int64_t)p.tiles * p.parts;
            local = atomicAdd(&cnt[p.cls], (int32_t)p.items);
        }
    }
    __syncthreads();
    if (threadIdx.x < kNumClasses) {
        int k = threadIdx.x;
        bbase[k] = cnt[k] ? atomicAdd(&ws->class_fill[k], cnt[k]) : 0;
    }
    __syncthreads();
    if (p.items > 0 && !ws->overflow) {
        const int64_t base = (int64_t)ws->class_base[p.cls] + bbase[p.cls] + local;
        if (base + p.items <= item_capacity) {
            const int b = n_boxes > 1 ? box_of_cell(boxes, n_boxes, (int32_t)c) : 0;
            // part-major: consecutive items are the tiles of one source part, so the waves that take them
            // together (one queue block goes to one XCD) stream the same sources through that XCD's L2
            int64_t k = base;
            for (int q = 0; q < p.parts; q++)
                for (int t = 0; t < p.tiles; t++) items[k++] = Item{(int32_t)c, t, q, b};
        }
    }
}

// ---------------------------------------------------------------- the force kernel

struct KArgs {
    const float4 *spos;
    const int32_t *cs;
    const int32_t *perm;
    const Item *items;
    WorkState *ws;
    const BoxDev *boxes;
    const ForceBox *fbox;
    const int32_t *cell_parts;
    const int64_t *cell_pbase;
    double *partials;
    float *acc;
    double *acc64;  // FP64 accelerations instead of acc when not null
    float *rho;
    unsigned long long *amax;   // [n_cells] bits of the largest |a|^2 written in each cell
    int R;
    int chunk;      // sources per LDS chunk
    int max_lanes;
    int region;     // bytes of LDS per wave
};

struct Seg {
    int32_t src, len, flat;
    float czref;
};

// Orders LDS traffic between the lanes of one wave (no other wave takes part).
__device__ inline void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

__device__ inline int sgpr(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Plummer pair term: g = (r2 + eps2)^(-3/2), with r2 = |d|^2 + eps2 returned.
__device__ __forceinline__ float plummer_g(float dx, float dy, float dz, float e2, float &r2) {
    r2 = __builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, __builtin_fmaf(dz, dz, e2)));
    const float ri = __builtin_amdgcn_rsqf(r2);
    const float ri2 = ri * ri;
    return ri2 * ri;
}

// Knuth's two-sum: s + e == a + b exactly.
__device__ __forceinline__ void two_sum(float a, float b, float &s, float &e) {
    s = a + b;
    const float bp = s - a;
    e = (a - (s - bp)) + (b - bp);
}

// |a|^2 of a written acceleration: FP64 squares of the stored values, each rounded, summed in a fixed order.
__device__ inline double norm2_written(double x, double y, double z) {
#pragma clang fp contract(off)
    return x * x + y * y + z * z;
}

// Largest |a|^2 of a cell: the bit patterns of non-negative doubles order like their values, so an
// integer maximum is exact and independent of the order of the updates.
__device__ inline void cell_max(unsigned long long *amax, int c, double v) {
    atomicMax(amax + c, (unsigned long long)__double_as_longlong(v));
}

__device__ inline double wave_max_f64(double v) {
    for (int off = 32; off > 0; off >>= 1) {
        const double y = __shfl_xor(v, off);
        v = v > y ? v : y;
    }
    return v;
}

// U staged sources against the S sinks of this lane.  With KDE, also the
// density weight max(0, 1 - r^2/b^2) = max(0, kc - r2 * ib2) (r2 carries the
// pair chain's constant offset, folded into kc).
template <int KIND, int MODE, int S, int U, bool KDE>
__device__ __forceinline__ void accumulate(const float4 (&p)[U], const float (&xi)[S], const float (&yi)[S],
                                           const float (&zi)[S], float c0, float c1, float c2, float e2,
                                           float ib2, float kc, float (&ax)[S], float (&ay)[S], float (&az)[S],
                                           double (&dxs)[S], double (&dys)[S], double (&dzs)[S], float (&rh)[S]) {
#pragma unroll
    for (int u = 0; u < U; u++) {
        float dx[S], dy[S], dz[S], r2[S], gg[S];
        if constexpr (KIND == ABACUS_NF_SPLINE) {
            // Spline: g = min(r^-3, c0 + r^2 (c1 r^-1 + c2)).  The cubic force polynomial (divided by r) lies
            // below r^-3 inside eps and above it outside, so the minimum selects the right branch without a
            // compare.  Newtonian regime test for the whole wave: when no lane has a pair closer than eps for
            // this source, g = r^-3 exactly and the polynomial and the minimum are skipped (one wave-uniform
            // branch; close pairs are rare at the softening lengths of the method).  r^2 > 0, so the bit
            // patterns of r^2 order as unsigned integers like the values: one integer minimum per lane, one
            // compare.
            unsigned rmin = 0xffffffffu;
#pragma unroll
            for (int s = 0; s < S; s++) {
                dx[s] = p[u].x - xi[s];
                dy[s] = p[u].y - yi[s];
                dz[s] = p[u].z - zi[s];
                r2[s] = __builtin_fmaf(dx[s], dx[s], __builtin_fmaf(dy[s], dy[s], __builtin_fmaf(dz[s], dz[s], kTiny)));
                rmin = min(rmin, __float_as_uint(r2[s]));
            }
            float ri[S];
#pragma unroll
            for (int s = 0; s < S; s++) {
                ri[s] = __builtin_amdgcn_rsqf(r2[s]);
                gg[s] = (ri[s] * ri[s]) * ri[s];
            }
            // some pair of the wave inside eps: the polynomial branch
            if (__builtin_amdgcn_ballot_w64(rmin < __float_as_uint(e2))) {
#pragma unroll
                for (int s = 0; s < S; s++)
                    gg[s] = fminf(gg[s], __builtin_fmaf(r2[s], __builtin_fmaf(c1, ri[s], c2), c0));
            }
        } else {
#pragma unroll
            for (int s = 0; s < S; s++) {
                dx[s] = p[u].x - xi[s];
                dy[s] = p[u].y - yi[s];
                dz[s] = p[u].z - zi[s];
                gg[s] = plummer_g(dx[s], dy[s], dz[s], e2, r2[s]);
            }
        }
#pragma unroll
        for (int s = 0; s < S; s++) {
            if constexpr (KDE) rh[s] += fmaxf(__builtin_fmaf(-r2[s], ib2, kc), 0.f);
            if constexpr (MODE == ABACUS_NF_SUM_FP64) {
                dxs[s] += (double)(dx[s] * gg[s]);
                dys[s] += (double)(dy[s] * gg[s]);
                dzs[s] += (double)(dz[s] * gg[s]);
            } else {
                ax[s] = __builtin_fmaf(dx[s], gg[s], ax[s]);
                ay[s] = __builtin_fmaf(dy[s], gg[s], ay[s]);
                az[s] = __builtin_fmaf(dz[s], gg[s], az[s]);
            }
        }
    }
}

// OCC > 0 asks the compiler for at least OCC waves per SIMD (a register budget of
// 512/OCC VGPRs); OCC = 0 leaves the register budget to the compiler.
template <int KIND, int MODE, int S, int U, int OCC, bool KDE>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(OCC > 0 ? OCC : 1, OCC > 0 ? OCC : 8)))
void k_forces(KArgs a) {
    constexpr int NC = KDE ? 4 : 3;  // reduced components per sink: acceleration (+ density)
    extern __shared__ __align__(16) unsigned char smem[];
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    unsigned char *region = smem + (size_t)wave * a.region;
    float4 *stage = (float4 *)region;
    Seg *segs = (Seg *)(region + (size_t)a.chunk * sizeof(float4));
    double *red = (double *)region;
    float *redf = (float *)region;
    const int R = a.R;
    const int W = 2 * R + 1;
    const int ncol = W * W;
    const int n_items = a.ws->n_items;
    const int home = blockIdx.x % kQueues;
    int queue = 0;  // queues tried so far (own queue first, then the others in turn)

    int jnext = 0, jleft = 0;   // slots of the current queue claimed and not yet taken: [jnext, jnext + jleft)
    for (;;) {
        // next item: slot j of queue x holds item x + kQueues*(j / kQueueBlock) (block) of the list; one atomic
        // claims one slot, or kLightClaim slots once the queue has reached its light items
        int k = n_items;
        while (queue < kQueues) {
            const int x = (home + queue) % kQueues;
            if (jleft == 0) {
                const int want = jnext >= a.ws->light_slot[x] ? kLightClaim : 1;
                int j = 0;
                if (lane == 0) j = atomicAdd(&a.ws->cursor[x], want);
                jnext = sgpr(__shfl(j, 0));
                jleft = want;
            }
            const int j = jnext;
            jnext++;
            jleft--;
            const int64_t idx = ((int64_t)(j / kQueueBlock) * kQueues + x) * kQueueBlock + j % kQueueBlock;
            if (idx < n_items) {
                k = (int)idx;
                break;
            }
            queue++;  // queue x is drained (its later slots only grow)
            jnext = 0;
            jleft = 0;
        }
        if (k >= n_items) break;
        const Item it = a.items[k];
        const int c = sgpr(it.cell);
        const int ib = sgpr(it.box);
        const BoxDev B = a.boxes[ib];
        const ForceBox F = a.fbox[ib];
        const int K = B.K;
        const int lin = c - B.cell_base;
        const int cz = lin % K, cy = (lin / K) % K, cx = lin / (K * K);
        const int cs0 = a.cs[c];
        const int nc = a.cs[c + 1] - cs0;
        const TileGeom tg = tile_at(nc, S, a.max_lanes, sgpr(it.tile));
        const int L = tg.L, G = tg.G;
        const int t0 = tg.t0;
        const int nt = tg.nt;
        const int g = lane / L, sub = lane - g * L;

        // sink tile: S sinks per lane, relative to the sink cell centre
        float xi[S], yi[S], zi[S];
#pragma unroll
        for (int s = 0; s < S; s++) {
            const int idx = g * S + s;
            float4 p = make_float4(0.f, 0.f, 0.f, 0.f);
            if (g < G && idx < nt) p = a.spos[cs0 + t0 + idx];
            xi[s] = p.x;
            yi[s] = p.y;
            zi[s] = p.z;
        }

        // segment table of the near field (one column per lane), flattened by a prefix sum
        ColSeg o;
        o.src0 = o.len0 = o.src1 = o.len1 = 0;
        o.czref0 = o.czref1 = 0.f;
        if (lane < ncol) {
            const int ex = wrap(cx + lane / W - R, K), ey = wrap(cy + lane % W - R, K);
            column_segments(a.cs, B.cell_base + (ex * K + ey) * K, cz, K, R, o);
        }
        int incl = o.len0 + o.len1;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const int y = __shfl_up(incl, off);
            if (lane >= off) incl += y;
        }
        const int nsrc = sgpr(__shfl(incl, 63));
        wave_lds_sync();
        if (lane < ncol) {
            const int start = incl - (o.len0 + o.len1);
            segs[2 * lane] = Seg{o.src0, o.len0, start, o.czref0};
            segs[2 * lane + 1] = Seg{o.src1, o.len1, start + o.len0, o.czref1};
        }
        wave_lds_sync();

        const int P = a.cell_parts[c];
        const int part = sgpr(it.part);
        // part boundaries: nsrc split into P near-equal contiguous ranges (32-bit arithmetic)
        const int pq = nsrc / P, pr = nsrc - pq * P;
        const int j0 = part * pq + min(part, pr);
        const int j1 = j0 + pq + (part < pr ? 1 : 0);

        float ax[S], ay[S], az[S];
        float hx[S], hy[S], hz[S], lx[S], ly[S], lz[S];
        double dxs[S], dys[S], dzs[S];
        float rh[S];
        double rhd[S];
#pragma unroll
        for (int s = 0; s < S; s++) {
            ax[s] = ay[s] = az[s] = 0.f;
            hx[s] = hy[s] = hz[s] = lx[s] = ly[s] = lz[s] = 0.f;
            dxs[s] = dys[s] = dzs[s] = 0.0;
            rh[s] = 0.f;
            rhd[s] = 0.0;
        }
        const float c0 = F.c0, c1 = F.c1, c2 = F.c2, e2 = F.eps2;
        const float ib2 = F.kde_ib2, kc = F.kde_c;
        const int step = L * U;
        const int nmax = (a.chunk / step) * step;

        int si = 0;
        for (int f = j0; f < j1;) {
            const int n = min(nmax, j1 - f);
            // stage [f, f+n) of the flattened source list, offsets applied
            int ff = f;
            while (ff < f + n) {
                Seg sg = segs[si];
                int sflat = sgpr(sg.flat), slen = sgpr(sg.len);
                while (sflat + slen <= ff && si + 1 < 2 * ncol) {
                    si++;
                    sg = segs[si];
                    sflat = sgpr(sg.flat);
                    slen = sgpr(sg.len);
                }
                const int end = min(sflat + slen, f + n);
                if (end <= ff) break;  // unreachable for a consistent table; guarantees termination
                const int col = si >> 1;
                const float offx = (float)(col / W - R), offy = (float)(col % W - R);
                const float czref = __builtin_bit_cast(float, sgpr(__builtin_bit_cast(int, sg.czref)));
                const int srcb = sgpr(sg.src) + (ff - sflat);
                const int cnt = end - ff;
                float4 *dst = stage + (ff - f);
                for (int q = lane; q < cnt; q += 64) {
                    const float4 p = a.spos[srcb + q];
                    dst[q] = make_float4(p.x + offx, p.y + offy, p.z + (p.w - czref), 0.f);
                }
                ff = end;
            }
            const int npad = ((n + step - 1) / step) * step;
            for (int q = n + lane; q < npad; q += 64) stage[q] = make_float4(kFar, kFar, kFar, 0.f);
            wave_lds_sync();

            if constexpr (MODE == ABACUS_NF_SUM_COMP32) {
#pragma unroll
                for (int s = 0; s < S; s++) ax[s] = ay[s] = az[s] = 0.f;
            }
            // uniform trip count; one sink group per lane (L == 1) reads with immediate LDS offsets
            const int iters = npad / step;
            if (L == 1) {
                const float4 *sp = stage;
                for (int it = 0; it < iters; ++it) {
                    float4 p[U];
#pragma unroll
                    for (int u = 0; u < U; u++) p[u] = sp[u];
                    sp += U;
                    accumulate<KIND, MODE, S, U, KDE>(p, xi, yi, zi, c0, c1, c2, e2, ib2, kc, ax, ay, az, dxs, dys,
                                                      dzs, rh);
                }
            } else {
                const float4 *sp = stage + sub;
                for (int it = 0; it < iters; ++it) {
                    float4 p[U];
#pragma unroll
                    for (int u = 0; u < U; u++) p[u] = sp[u * L];
                    sp += step;
                    accumulate<KIND, MODE, S, U, KDE>(p, xi, yi, zi, c0, c1, c2, e2, ib2, kc, ax, ay, az, dxs, dys,
                                                      dzs, rh);
                }
            }
            if constexpr (KDE && MODE != ABACUS_NF_SUM_FP32) {
#pragma unroll
                for (int s = 0; s < S; s++) {
                    rhd[s] += (double)rh[s];
                    rh[s] = 0.f;
                }
            }
            if constexpr (MODE == ABACUS_NF_SUM_COMP32) {
#pragma unroll
                for (int s = 0; s < S; s++) {
                    float e;
                    two_sum(hx[s], ax[s], hx[s], e);
                    lx[s] += e;
                    two_sum(hy[s], ay[s], hy[s], e);
                    ly[s] += e;
                    two_sum(hz[s], az[s], hz[s], e);
                    lz[s] += e;
                }
            }
            wave_lds_sync();
            f += n;
        }

        // ordered reduction over the L lanes that share each sink (all components at once)
#pragma unroll
        for (int s = 0; s < S; s++) {
            const int o = (lane * S + s) * NC;
            if constexpr (MODE == ABACUS_NF_SUM_FP32) {
                redf[o + 0] = ax[s];
                redf[o + 1] = ay[s];
                redf[o + 2] = az[s];
                if constexpr (KDE) redf[o + 3] = rh[s];
            } else if constexpr (MODE == ABACUS_NF_SUM_COMP32) {
                red[o + 0] = (double)hx[s] + (double)lx[s];
                red[o + 1] = (double)hy[s] + (double)ly[s];
                red[o + 2] = (double)hz[s] + (double)lz[s];
                if constexpr (KDE) red[o + 3] = rhd[s];
            } else {
                red[o + 0] = dxs[s];
                red[o + 1] = dys[s];
                red[o + 2] = dzs[s];
                if constexpr (KDE) red[o + 3] = rhd[s];
            }
        }
        wave_lds_sync();
        double amax2 = 0.0;   // largest |a|^2 this lane writes (cells written here, not split ones)
        if (sub == 0 && g < G) {
            const bool split = P > 1;
            for (int s = 0; s < S; s++) {
                const int idx = g * S + s;
                if (idx >= nt) break;
                const int base = (g * L * S + s) * NC;
                if (!split) {
                    const int64_t i = a.perm[cs0 + t0 + idx];
                    double w[3];   // the values written
                    for (int d = 0; d < NC; d++) {
                        double v;   // the value before its (optional) rounding to FP32
                        if constexpr (MODE == ABACUS_NF_SUM_FP32) {
                            float t = 0.f;
                            for (int q = 0; q < L; q++) t += redf[base + q * S * NC + d];
                            v = d < 3 ? t * F.scalef : t;
                        } else {
                            double t = 0.0;
                            for (int q = 0; q < L; q++) t += red[base + q * S * NC + d];
                            v = d < 3 ? t * F.scale : t;
                        }
                        if (d == 3) {
                            a.rho[i] = (float)v;
                        } else if (a.acc64) {
                            a.acc64[3 * i + d] = v;
                            w[d] = v;
                        } else {
                            a.acc[3 * i + d] = (float)v;
                            w[d] = (double)(float)v;
                        }
                    }
                    const double m = norm2_written(w[0], w[1], w[2]);
                    amax2 = m > amax2 ? m : amax2;
                } else {
                    double *out = a.partials + (int64_t)NC * (a.cell_pbase[c] + (int64_t)part * nc + t0 + idx);
                    for (int d = 0; d < NC; d++) {
                        if constexpr (MODE == ABACUS_NF_SUM_FP32) {
                            float t = 0.f;
                            for (int q = 0; q < L; q++) t += redf[base + q * S * NC + d];
                            out[d] = t;
                        } else {
                            double t = 0.0;
                            for (int q = 0; q < L; q++) t += red[base + q * S * NC + d];
                            out[d] = t;
                        }
                    }
                }
            }
        }
        if (P <= 1) {   // per-cell maximum of |a|^2 (the input of the step-size criterion)
            amax2 = wave_max_f64(amax2);
            if (lane == 0 && amax2 > 0.0) cell_max(a.amax, c, amax2);
        }
        wave_lds_sync();
    }
}

// Sinks whose source list was split: add the parts in order and write the result.
template <int MODE, int NC>
__global__ __launch_bounds__(256) void k_finalize(const WorkState *__restrict__ ws, int64_t partial_capacity,
                                                  const int32_t *__restrict__ keys, const int32_t *__restrict__ cs,
                                                  const int32_t *__restrict__ perm,
                                                  const int32_t *__restrict__ cell_parts,
                                                  const int64_t *__restrict__ cell_pbase,
                                                  const double *__restrict__ partials,
                                                  const BoxDev *__restrict__ boxes, int n_boxes,
                                                  const ForceBox *__restrict__ fbox, float *__restrict__ acc,
                                                  double *__restrict__ acc64, float *__restrict__ rho,
                                                  unsigned long long *__restrict__ amax, int64_t n) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (ws->overflow) return;
    const int lane = threadIdx.x & 63;
    int32_t c = -1;
    double m = 0.0;   // |a|^2 written for this slot
    if (s < n) {
        c = keys[s];
        const int P = cell_parts[c];
        const int cs0 = cs[c], nc = cs[c + 1] - cs0;
        const int64_t base = cell_pbase[c] + (s - cs0);
        if (P > 1 && base + (int64_t)(P - 1) * nc < partial_capacity) {
            const int b = n_boxes > 1 ? box_of_cell(boxes, n_boxes, c) : 0;
            const ForceBox F = fbox[b];
            const int64_t i = perm[s];
            double w[3];
            for (int d = 0; d < NC; d++) {
                double v;   // the value before its (optional) rounding to FP32
                if constexpr (MODE == ABACUS_NF_SUM_FP32) {
                    float t = 0.f;
                    for (int p = 0; p < P; p++) t += (float)partials[NC * (base + (int64_t)p * nc) + d];
                    v = d < 3 ? t * F.scalef : t;
                } else {
                    double t = 0.0;
                    for (int p = 0; p < P; p++) t += partials[NC * (base + (int64_t)p * nc) + d];
                    v = d < 3 ? t * F.scale : t;
                }
                if (d == 3) {
                    rho[i] = (float)v;
                } else if (acc64) {
                    acc64[3 * i + d] = v;
                    w[d] = v;
                } else {
                    acc[3 * i + d] = (float)v;
                    w[d] = (double)(float)v;
                }
            }
            m = norm2_written(w[0], w[1], w[2]);
        }
    }
    // per-cell maximum over the wave's slots: a segmented max-scan (slots are sorted by cell, so equal
    // keys are adjacent) and one update by the last lane of each run
    for (int off = 1; off < 64; off <<= 1) {
        const double y = __shfl_up(m, off);
        const int cy = __shfl_up(c, off);
        if (lane >= off && cy == c) m = m > y ? m : y;
    }
    const int cn = __shfl_down(c, 1);
    if (c >= 0 && m > 0.0 && (lane == 63 || cn != c)) cell_max(amax, c, m);
}

// ---------------------------------------------------------------- variant dispatch

typedef void (*ForcesKernel)(KArgs);

template <int KIND, int MODE, int S, int U, bool KDE>
ForcesKernel pick_occ(int occ) {
    if constexpr (KDE) {  // density variants: compiler's register budget, 6 or 8 waves per SIMD
        switch (occ) {
            case 6: return k_forces<KIND, MODE, S, U, 6, true>;
            case 8: return k_forces<KIND, MODE, S, U, 8, true>;
            default: return k_forces<KIND, MODE, S, U, 0, true>;
        }
    } else {
        switch (occ) {
            case 6: return k_forces<KIND, MODE, S, U, 6, false>;
            case 8: return k_forces<KIND, MODE, S, U, 8, false>;
            default: return k_forces<KIND, MODE, S, U, 0, false>;
        }
    }
}

template <int KIND, int MODE, int S, bool KDE>
ForcesKernel pick_u(int U, int occ) {
    switch (U) {
        case 1: return pick_occ<KIND, MODE, S, 1, KDE>(occ);
        case 4:
            if constexpr (!KDE) return pick_occ<KIND, MODE, S, 4, KDE>(occ);
            else return pick_occ<KIND, MODE, S, 2, KDE>(occ);
        default: return pick_occ<KIND, MODE, S, 2, KDE>(occ);
    }
}

template <int KIND, int MODE, bool KDE>
ForcesKernel pick_s(int S, int U, int occ) {
    switch (S) {
        case 1: return pick_u<KIND, MODE, 1, KDE>(U, occ);
        case 4: return pick_u<KIND, MODE, 4, KDE>(U, occ);
        default: return pick_u<KIND, MODE, 2, KDE>(U, occ);
    }
}

template <int KIND, bool KDE>
ForcesKernel pick_mode(int mode, int S, int U, int occ) {
    switch (mode) {
        case ABACUS_NF_SUM_COMP32: return pick_s<KIND, ABACUS_NF_SUM_COMP32, KDE>(S, U, occ);
        case ABACUS_NF_SUM_FP64: return pick_s<KIND, ABACUS_NF_SUM_FP64, KDE>(S, U, occ);
        default: return pick_s<KIND, ABACUS_NF_SUM_FP32, KDE>(S, U, occ);
    }
}

ForcesKernel pick_kernel(abacus_nf_kind kind, abacus_nf_sum mode, int S, int U, int occ, bool kde) {
    if (kde)
        return kind == ABACUS_NF_PLUMMER ? pick_mode<ABACUS_NF_PLUMMER, true>(mode, S, U, occ)
                                         : pick_mode<ABACUS_NF_SPLINE, true>(mode, S, U, occ);
    return kind == ABACUS_NF_PLUMMER ? pick_mode<ABACUS_NF_PLUMMER, false>(mode, S, U, occ)
                                     : pick_mode<ABACUS_NF_SPLINE, false>(mode, S, U, occ);
}

size_t region_bytes(const abacus_nf_tuning &t) {
    size_t stage = (size_t)t.chunk * sizeof(float4);
    size_t red = (size_t)64 * t.sinks_per_lane * 4 * sizeof(double);
    size_t main = stage > red ? stage : red;
    return (main + (size_t)2 * 49 * sizeof(Seg) + 15) & ~(size_t)15;
}

}  // namespace

// ---------------------------------------------------------------- host side

hipError_t launch_set_force_boxes(const double *eps, const double *gm, const double *kde_b, abacus_nf_kind kind,
                                  const abacus_nf_box *boxes, int n_boxes, ForceBox *dst, hipStream_t st) {
    for (int first = 0; first < n_boxes; first += kFBoxChunk) {
        FBoxChunk ch;
        memset(&ch, 0, sizeof(ch));
        ch.first = first;
        ch.count = n_boxes - first < kFBoxChunk ? n_boxes - first : kFBoxChunk;
        for (int k = 0; k < ch.count; k++) {
            const int b = first + k;
            const double w = boxes[b].box / boxes[b].K;
            const double e = eps[b] / w;
            ForceBox &f = ch.f[k];
            f.c0 = (float)(10.0 / (e * e * e));
            f.c1 = (float)(-15.0 / (e * e * e * e));
            f.c2 = (float)(6.0 / (e * e * e * e * e));
            f.eps2 = (float)(e * e);
            f.scale = gm[b] / (w * w);
            f.scalef = (float)f.scale;
            if (kde_b) {
                const double bc = kde_b[b] / w;
                const double ib2 = 1.0 / (bc * bc);
                const double offset = kind == ABACUS_NF_PLUMMER ? (double)f.eps2 : (double)kTiny;
                f.kde_ib2 = (float)ib2;
                f.kde_c = (float)(1.0 + offset * ib2);
            } else {
                f.kde_ib2 = 0.f;
                f.kde_c = 0.f;
            }
            f.pad = 0;
        }
        hipLaunchKernelGGL(k_set_fbox, dim3(1), dim3(kFBoxChunk), 0, st, ch, dst);
        hipError_t err = hipGetLastError();
        if (err != hipSuccess) return err;
    }
    return hipSuccess;
}

hipError_t launch_count_interactions(const ForcesArgs &a, hipStream_t st) {
    hipLaunchKernelGGL(k_wl_clear, dim3(1), dim3(kNumClasses), 0, st, a.ws, a.tune.part_sources);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || a.n_cells <= 0) return e;
    hipLaunchKernelGGL(k_wl_cells, dim3(grid_for(a.n_cells, 256)), dim3(256), 0, st, a.cell_start, a.boxes,
                       a.n_boxes, a.n_cells, a.R, a.tune.sinks_per_lane, a.tune.max_lanes, a.cell_nsrc, a.ws);
    return hipGetLastError();
}

hipError_t build_work_list(const ForcesArgs &a, hipStream_t st) {
    hipError_t e = launch_count_interactions(a, st);
    if (e != hipSuccess || a.n_cells <= 0) return e;
    if ((e = launch_fill_u64(a.amax, a.n_cells, 0ull, st)) != hipSuccess) return e;
    const int S = a.tune.sinks_per_lane, ML = a.tune.max_lanes;
    const unsigned gc = grid_for(a.n_cells, 256);
    hipLaunchKernelGGL(k_wl_plan, dim3(1), dim3(64), 0, st, a.ws, a.partial_capacity, a.item_capacity, a.n_total);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_wl_count, dim3(gc), dim3(256), 0, st, a.cell_start, a.cell_nsrc, a.n_cells, S, ML, a.ws,
                       a.cell_parts, a.cell_pdem);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    e = scan_i64_add_exclusive(a.cell_pdem, a.cell_pbase, a.n_cells, a.scan_temp, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_wl_classes, dim3(1), dim3(64), 0, st, a.ws, a.item_capacity, a.cell_pbase, a.cell_pdem,
                       a.n_cells, a.partial_capacity, a.err);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_wl_emit, dim3(gc), dim3(256), 0, st, a.cell_start, a.cell_nsrc, a.cell_parts, a.boxes,
                       a.n_boxes, a.n_cells, S, ML, a.ws, a.items, a.item_capacity);
    return hipGetLastError();
}

int forces_grid(const abacus_nf_tuning &t, abacus_nf_kind kind, abacus_nf_sum mode, bool kde, int device) {
    ForcesKernel kfn = pick_kernel(kind, mode, t.sinks_per_lane, t.unroll, t.occupancy, kde);
    const size_t lds = region_bytes(t) * kWaves;
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)kfn, kThreads, lds) != hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    if (t.waves_per_cu > 0) {
        int want = (t.waves_per_cu + kWaves - 1) / kWaves;
        if (want < per_cu) per_cu = want;
    }
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || cus < 1) cus = 1;
    return per_cu * cus;
}

hipError_t launch_forces(const ForcesArgs &a, hipStream_t st) {
    if (a.n_total <= 0) return hipSuccess;
    KArgs k;
    k.spos = a.spos;
    k.cs = a.cell_start;
    k.perm = a.perm;
    k.items = a.items;
    k.ws = a.ws;
    k.boxes = a.boxes;
    k.fbox = a.fbox;
    k.cell_parts = a.cell_parts;
    k.cell_pbase = a.cell_pbase;
    k.partials = a.partials;
    k.acc = a.acc;
    k.acc64 = a.acc64;
    k.rho = a.rho;
    k.amax = a.amax;
    k.R = a.R;
    k.chunk = a.tune.chunk;
    k.max_lanes = a.tune.max_lanes;
    k.region = (int)region_bytes(a.tune);
    ForcesKernel kfn = pick_kernel(a.kind, a.mode, a.tune.sinks_per_lane, a.tune.unroll, a.tune.occupancy,
                                   a.rho != nullptr);
    hipLaunchKernelGGL(kfn, dim3(a.grid), dim3(kThreads), (size_t)k.region * kWaves, st, k);
    return hipGetLastError();
}

hipError_t launch_finalize(const ForcesArgs &a, hipStream_t st) {
    if (a.n_total <= 0) return hipSuccess;
    const unsigned gn = grid_for(a.n_total, 256);
    const bool f32 = a.mode == ABACUS_NF_SUM_FP32, kde = a.rho != nullptr;
    auto kfn = f32 ? (kde ? k_finalize<ABACUS_NF_SUM_FP32, 4> : k_finalize<ABACUS_NF_SUM_FP32, 3>)
                   : (kde ? k_finalize<ABACUS_NF_SUM_FP64, 4> : k_finalize<ABACUS_NF_SUM_FP64, 3>);
    hipLaunchKernelGGL(kfn, dim3(gn), dim3(256), 0, st, a.ws, a.partial_capacity, a.keys, a.cell_start, a.perm,
                       a.cell_parts, a.cell_pbase, a.partials, a.boxes, a.n_boxes, a.fbox, a.acc, a.acc64, a.rho,
                       a.amax, a.n_total);
    return hipGetLastError();
}

}  // namespace anf

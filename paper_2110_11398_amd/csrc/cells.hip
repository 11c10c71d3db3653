// Cell construction for the near-field force: binning, a stable LSD radix sort
// of particles by cell, the cell offsets, and the cell-relative FP32 layout.
//
// Sec. 3.1 of the paper cuts each periodic box into a cubic lattice of CPD^3
// cells; the near field of a particle is defined by the cells around its own.
// The paper's CPU pipeline re-bins particles and transposes positions for the
// GPU every step (Table "tbl:timing": "Transpose Positions", "Merge New
// Particles").  Here the equivalent is done on the device, in HBM:
//
//   k_bin            cell of every particle (FP64 cell rule), key/value pairs
//   k_radix_hist     per-tile digit histograms of the keys          } one pass per
//   scan             exclusive scan of the (digit, tile) counts      } 8-bit digit,
//   k_radix_scatter  stable scatter (wave ballots rank equal digits) } LSD order
//   k_run_ends       end slot of every non-empty cell; a max-scan turns those
//                    into the cell offsets (empty cells inherit the previous end)
//   k_gather         cell-relative coordinates in cell widths, FP64 -> FP32
//
// Every step is deterministic: particles of a cell stay in input order.
#include <cstring>

#include "nf_internal.h"

namespace anf {

namespace {

constexpr int kTileThreads = 256;
constexpr int kTileItems = 16;
constexpr int kTile = kTileThreads * kTileItems;  // 4096 elements per workgroup

inline unsigned grid_for(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

// ---------------------------------------------------------------- fills / boxes

__global__ void k_fill_i32(int32_t *p, int64_t n, int32_t v) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

constexpr int kBoxChunk = 24;
struct BoxChunk {
    BoxDev b[kBoxChunk];
    int first, count;
};

__global__ void k_set_boxes(BoxChunk c, BoxDev *dst) {
    int i = threadIdx.x;
    if (i < c.count) dst[c.first + i] = c.b[i];
}

// The cell rule along one axis, every FP64 operation rounded on its own:
//   xt = x - L*floor(x/L),  t = xt*s (s = K/L),  c = min(floor(t), K-1).
__device__ inline int axis_cell(double x, double L, double s, int K, double *t_out) {
#pragma clang fp contract(off)
    double q = floor(x / L);
    double xt = x - L * q;
    double t = xt * s;
    double f = floor(t);
    int c = (f >= (double)(K - 1)) ? (K - 1) : (int)f;
    if (c < 0) c = 0;
    *t_out = t;
    return c;
}

__global__ __launch_bounds__(256) void k_bin(const float *__restrict__ pos, int64_t n,
                                             const BoxDev *__restrict__ boxes, int n_boxes,
                                             int32_t *__restrict__ keys, int32_t *__restrict__ vals, int *err) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int b = n_boxes > 1 ? box_of_particle(boxes, n_boxes, i) : 0;
    const BoxDev B = boxes[b];
    double x = pos[3 * i], y = pos[3 * i + 1], z = pos[3 * i + 2];
    int32_t key = B.cell_base;
    if (isfinite(x) && isfinite(y) && isfinite(z)) {
        double t;
        int cx = axis_cell(x, B.L, B.s, B.K, &t);
        int cy = axis_cell(y, B.L, B.s, B.K, &t);
        int cz = axis_cell(z, B.L, B.s, B.K, &t);
        key = B.cell_base + (cx * B.K + cy) * B.K + cz;
    } else {
        atomicCAS(err, 0, ABACUS_NF_ENONFINITE);
    }
    keys[i] = key;
    vals[i] = (int32_t)i;
}

// ---------------------------------------------------------------- scans

struct OpAdd {
    template <typename T> __device__ T operator()(T a, T b) const { return a + b; }
};
struct OpMax {
    template <typename T> __device__ T operator()(T a, T b) const { return a > b ? a : b; }
};

// Scan of one tile of kTile elements: each thread scans 16 consecutive
// elements, a Hillis-Steele pass over the 256 thread totals adds the prefix.
template <typename T, typename Op>
__global__ __launch_bounds__(kTileThreads) void k_scan_tile(const T *in, T *out, T *sums, int64_t n, int inclusive,
                                                           T identity) {
    __shared__ T s[kTileThreads];
    Op op;
    int tid = threadIdx.x;
    int64_t base = (int64_t)blockIdx.x * kTile + (int64_t)tid * kTileItems;
    T v[kTileItems];
    T run = identity;
#pragma unroll
    for (int k = 0; k < kTileItems; k++) {
        int64_t i = base + k;
        T x = i < n ? in[i] : identity;
        T nr = op(run, x);
        v[k] = inclusive ? nr : run;
        run = nr;
    }
    s[tid] = run;
    __syncthreads();
    for (int off = 1; off < kTileThreads; off <<= 1) {
        T y = tid >= off ? s[tid - off] : identity;
        __syncthreads();
        s[tid] = op(s[tid], y);
        __syncthreads();
    }
    T prefix = tid > 0 ? s[tid - 1] : identity;
#pragma unroll
    for (int k = 0; k < kTileItems; k++) {
        int64_t i = base + k;
        if (i < n) out[i] = op(prefix, v[k]);
    }
    if (sums && tid == kTileThreads - 1) sums[blockIdx.x] = s[kTileThreads - 1];
}

template <typename T, typename Op>
__global__ void k_scan_add(T *out, const T *offs, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        int64_t b = i / kTile;
        if (b > 0) out[i] = Op()(offs[b], out[i]);
    }
}

size_t scan_levels_bytes(int64_t n, size_t elem) {
    size_t bytes = 0;
    while (n > kTile) {
        int64_t nt = (n + kTile - 1) / kTile;
        bytes += 2 * (size_t)nt * elem + 256;
        n = nt;
    }
    return bytes;
}

template <typename T, typename Op>
hipError_t scan_impl(const T *in, T *out, int64_t n, bool inclusive, T identity, char *temp, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    int64_t nt = (n + kTile - 1) / kTile;
    if (nt == 1) {
        hipLaunchKernelGGL((k_scan_tile<T, Op>), dim3(1), dim3(kTileThreads), 0, st, in, out, (T *)nullptr, n,
                           (int)inclusive, identity);
        return hipGetLastError();
    }
    T *sums = (T *)temp;
    T *offs = sums + nt;
    char *next = (char *)(((uintptr_t)(offs + nt) + 255) & ~(uintptr_t)255);
    hipLaunchKernelGGL((k_scan_tile<T, Op>), dim3((unsigned)nt), dim3(kTileThreads), 0, st, in, out, sums, n,
                       (int)inclusive, identity);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = scan_impl<T, Op>(sums, offs, nt, false, identity, next, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_scan_add<T, Op>), dim3(grid_for(n, 256)), dim3(256), 0, st, out, offs, n);
    return hipGetLastError();
}

// ---------------------------------------------------------------- radix sort

constexpr int kRadixMaxBits = 8;
constexpr int kRadixBins = 1 << kRadixMaxBits;
constexpr int kWaveSpan = kTile / 4;  // contiguous elements handled by one wave of a tile

__global__ __launch_bounds__(kTileThreads) void k_radix_hist(const int32_t *__restrict__ keys, int64_t n, int shift,
                                                             int bits, uint32_t *__restrict__ thist, int ntiles) {
    __shared__ uint32_t h[kRadixBins];
    int tid = threadIdx.x;
    h[tid] = 0;
    __syncthreads();
    int64_t base = (int64_t)blockIdx.x * kTile;
    uint32_t mask = (1u << bits) - 1u;
#pragma unroll 4
    for (int k = 0; k < kTileItems; k++) {
        int64_t i = base + (int64_t)k * kTileThreads + tid;
        if (i < n) atomicAdd(&h[((uint32_t)keys[i] >> shift) & mask], 1u);
    }
    __syncthreads();
    if (tid < (1 << bits)) thist[(int64_t)tid * ntiles + blockIdx.x] = h[tid];
}

// Stable scatter of one tile.  Wave w owns the contiguous span
// [tile + w*1024, tile + (w+1)*1024), read in 16 rounds of 64.  Within a
// round, lanes with equal digits are found with one ballot per digit bit; a
// lane's rank is the number of equal lanes below it plus the wave's running
// count of that digit.  Wave counts are then prefix-summed across the four
// waves, and the tile's digit totals across the digits: every element gets
// its position in the tile sorted by digit (input order within a digit).  The
// tile is staged in LDS in that order and written out by consecutive threads,
// so each digit's run goes to global memory in whole, contiguous pieces at
// the tile's global offset for the digit (from the scanned (digit, tile)
// histogram).
__global__ __launch_bounds__(kTileThreads) void k_radix_scatter(const int32_t *__restrict__ kin,
                                                                const int32_t *__restrict__ vin,
                                                                int32_t *__restrict__ kout,
                                                                int32_t *__restrict__ vout, int64_t n, int shift,
                                                                int bits, const uint32_t *__restrict__ toff,
                                                                int ntiles) {
    static_assert(kTileThreads == kRadixBins, "one thread per digit in the per-digit steps");
    __shared__ uint32_t wcnt[4][kRadixBins];
    __shared__ uint32_t goff[kRadixBins];
    __shared__ uint32_t loff[kRadixBins];
    __shared__ int32_t skey[kTile];
    __shared__ int32_t sval[kTile];
    int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    for (int d = tid; d < 4 * kRadixBins; d += kTileThreads) (&wcnt[0][0])[d] = 0;
    if (tid < (1 << bits)) goff[tid] = toff[(int64_t)tid * ntiles + blockIdx.x];
    __syncthreads();
    const uint32_t mask = (1u << bits) - 1u;
    const uint64_t below_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const int64_t tile = (int64_t)blockIdx.x * kTile;
    const int64_t base = tile + (int64_t)w * kWaveSpan;
    int32_t key[kTileItems], val[kTileItems];
    uint32_t rank[kTileItems];
#pragma unroll
    for (int r = 0; r < kTileItems; r++) {
        int64_t i = base + (int64_t)r * 64 + lane;
        bool valid = i < n;
        key[r] = valid ? kin[i] : 0;
        val[r] = valid ? vin[i] : 0;
        uint32_t d = ((uint32_t)key[r] >> shift) & mask;
        uint64_t m = __ballot(valid);
        for (int b = 0; b < bits; b++) {
            int bit = (d >> b) & 1u;
            uint64_t bb = __ballot(bit);
            m &= bit ? bb : ~bb;
        }
        uint32_t below = (uint32_t)__popcll(m & below_mask);
        uint32_t cnt = (uint32_t)__popcll(m);
        uint32_t c0 = valid ? wcnt[w][d] : 0u;
        rank[r] = c0 + below;
        if (valid && below == 0) wcnt[w][d] = c0 + cnt;
    }
    __syncthreads();
    {
        // digit tid: prefix over the waves, and the tile's total
        uint32_t run = 0;
        for (int w2 = 0; w2 < 4; w2++) {
            uint32_t c = wcnt[w2][tid];
            wcnt[w2][tid] = run;
            run += c;
        }
        loff[tid] = run;
    }
    __syncthreads();
    if (w == 0) {
        // exclusive scan of the tile's digit totals: four digits per lane, then a wave scan of the lane sums
        uint32_t v[4], s = 0;
#pragma unroll
        for (int q = 0; q < 4; q++) {
            v[q] = s;
            s += loff[4 * lane + q];
        }
        uint32_t incl = s;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t y = __shfl_up(incl, off);
            if (lane >= off) incl += y;
        }
        const uint32_t excl = incl - s;
#pragma unroll
        for (int q = 0; q < 4; q++) loff[4 * lane + q] = excl + v[q];
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kTileItems; r++) {
        int64_t i = base + (int64_t)r * 64 + lane;
        if (i < n) {
            const uint32_t d = ((uint32_t)key[r] >> shift) & mask;
            const uint32_t lp = loff[d] + wcnt[w][d] + rank[r];
            skey[lp] = key[r];
            sval[lp] = val[r];
        }
    }
    __syncthreads();
    const int64_t left = n - tile;
    const int tile_n = left < kTile ? (int)left : kTile;
#pragma unroll 4
    for (int j = 0; j < kTileItems; j++) {
        const int lp = j * kTileThreads + tid;
        if (lp < tile_n) {
            const int32_t k = skey[lp];
            const uint32_t d = ((uint32_t)k >> shift) & mask;
            const uint32_t dest = goff[d] + ((uint32_t)lp - loff[d]);
            kout[dest] = k;
            vout[dest] = sval[lp];
        }
    }
}

// ---------------------------------------------------------------- cell offsets and layout

__global__ void k_run_ends(const int32_t *__restrict__ keys, int64_t n, int32_t *__restrict__ endpos) {
    int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    int32_t k = keys[s];
    if (s == n - 1 || keys[s + 1] != k) endpos[k] = (int32_t)(s + 1);
}

// spos[s] = (t_x - (c_x + 1/2), t_y - (c_y + 1/2), t_z - (c_z + 1/2), c_z) where
// t = xt*K/L is the wrapped coordinate in cell widths: positions relative to
// the centre of their own cell, in cell widths, rounded once to FP32.
__global__ __launch_bounds__(256) void k_gather(const float *__restrict__ pos, const int32_t *__restrict__ perm,
                                                const int32_t *__restrict__ keys, int64_t n,
                                                const BoxDev *__restrict__ boxes, int n_boxes,
                                                float4 *__restrict__ spos) {
    int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    int64_t i = perm[s];
    int b = n_boxes > 1 ? box_of_cell(boxes, n_boxes, keys[s]) : 0;
    const BoxDev B = boxes[b];
    double x = pos[3 * i], y = pos[3 * i + 1], z = pos[3 * i + 2];
    float4 o = make_float4(0.f, 0.f, 0.f, 0.f);
    if (isfinite(x) && isfinite(y) && isfinite(z)) {
        double tx, ty, tz;
        int cx = axis_cell(x, B.L, B.s, B.K, &tx);
        int cy = axis_cell(y, B.L, B.s, B.K, &ty);
        int cz = axis_cell(z, B.L, B.s, B.K, &tz);
        o.x = (float)(tx - ((double)cx + 0.5));
        o.y = (float)(ty - ((double)cy + 0.5));
        o.z = (float)(tz - ((double)cz + 0.5));
        o.w = (float)cz;
    }
    spos[s] = o;
}

}  // namespace

// ---------------------------------------------------------------- host launchers

hipError_t launch_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(n, 256)), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}

hipError_t launch_set_boxes(const abacus_nf_box *boxes, int n_boxes, const int32_t *cell_base, BoxDev *dst,
                            hipStream_t st) {
    for (int first = 0; first < n_boxes; first += kBoxChunk) {
        BoxChunk c;
        memset(&c, 0, sizeof(c));
        c.first = first;
        c.count = n_boxes - first < kBoxChunk ? n_boxes - first : kBoxChunk;
        for (int k = 0; k < c.count; k++) {
            const abacus_nf_box &b = boxes[first + k];
            c.b[k].offset = b.offset;
            c.b[k].n = b.n;
            c.b[k].L = b.box;
            c.b[k].s = (double)b.K / b.box;
            c.b[k].K = b.K;
            c.b[k].cell_base = cell_base[first + k];
        }
        hipLaunchKernelGGL(k_set_boxes, dim3(1), dim3(kBoxChunk), 0, st, c, dst);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_bin(const float *pos, int64_t n, const BoxDev *boxes, int n_boxes, int32_t *keys, int32_t *vals,
                      int *err, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_bin, dim3(grid_for(n, 256)), dim3(256), 0, st, pos, n, boxes, n_boxes, keys, vals, err);
    return hipGetLastError();
}

size_t scan_temp_bytes(int64_t n) { return scan_levels_bytes(n, sizeof(int64_t)) + 1024; }

hipError_t scan_i32_max_inclusive(const int32_t *in, int32_t *out, int64_t n, void *temp, hipStream_t st) {
    return scan_impl<int32_t, OpMax>(in, out, n, true, (int32_t)0, (char *)temp, st);
}

hipError_t scan_i64_add_exclusive(const int64_t *in, int64_t *out, int64_t n, void *temp, hipStream_t st) {
    return scan_impl<int64_t, OpAdd>(in, out, n, false, (int64_t)0, (char *)temp, st);
}

size_t radix_temp_bytes(int64_t n) {
    int64_t ntiles = (n + kTile - 1) / kTile;
    int64_t hist = ntiles * kRadixBins;
    return 2 * (size_t)hist * sizeof(uint32_t) + scan_levels_bytes(hist, sizeof(uint32_t)) + 1024;
}

hipError_t radix_sort_pairs(int32_t *keys, int32_t *vals, int32_t *keys_tmp, int32_t *vals_tmp, void *temp,
                            int64_t n, int key_bits, hipStream_t st, int32_t **keys_out, int32_t **vals_out) {
    *keys_out = keys;
    *vals_out = vals;
    if (n <= 1 || key_bits <= 0) return hipSuccess;
    int passes = (key_bits + kRadixMaxBits - 1) / kRadixMaxBits;
    int bits = (key_bits + passes - 1) / passes;
    int ntiles = (int)((n + kTile - 1) / kTile);
    int64_t hist = (int64_t)ntiles << bits;
    uint32_t *thist = (uint32_t *)temp;
    uint32_t *toff = thist + (size_t)ntiles * kRadixBins;
    char *scan_tmp = (char *)(((uintptr_t)(toff + (size_t)ntiles * kRadixBins) + 255) & ~(uintptr_t)255);
    int32_t *ka = keys, *va = vals, *kb = keys_tmp, *vb = vals_tmp;
    for (int p = 0, shift = 0; p < passes; p++, shift += bits) {
        int pb = (key_bits - shift) < bits ? (key_bits - shift) : bits;
        int64_t h = (int64_t)ntiles << pb;
        (void)hist;
        hipLaunchKernelGGL(k_radix_hist, dim3(ntiles), dim3(kTileThreads), 0, st, ka, n, shift, pb, thist, ntiles);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        e = scan_impl<uint32_t, OpAdd>(thist, toff, h, false, 0u, scan_tmp, st);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_radix_scatter, dim3(ntiles), dim3(kTileThreads), 0, st, ka, va, kb, vb, n, shift, pb,
                           toff, ntiles);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        int32_t *t;
        t = ka; ka = kb; kb = t;
        t = va; va = vb; vb = t;
    }
    *keys_out = ka;
    *vals_out = va;
    return hipSuccess;
}

hipError_t launch_cell_start(const int32_t *keys_sorted, int64_t n, int64_t n_cells, int32_t *endpos,
                             int32_t *cell_start, void *scan_temp, hipStream_t st) {
    hipError_t e = launch_fill_i32(endpos, n_cells, 0, st);
    if (e != hipSuccess) return e;
    e = launch_fill_i32(cell_start, 1, 0, st);
    if (e != hipSuccess) return e;
    if (n > 0) {
        hipLaunchKernelGGL(k_run_ends, dim3(grid_for(n, 256)), dim3(256), 0, st, keys_sorted, n, endpos);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return scan_i32_max_inclusive(endpos, cell_start + 1, n_cells, scan_temp, st);
}

hipError_t launch_gather(const float *pos, const int32_t *perm, const int32_t *keys_sorted, int64_t n,
                         const BoxDev *boxes, int n_boxes, float4 *spos, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather, dim3(grid_for(n, 256)), dim3(256), 0, st, pos, perm, keys_sorted, n, boxes,
                       n_boxes, spos);
    return hipGetLastError();
}

}  // namespace anf

// Leapfrog time stepping: kick, drift and the cell timestep criterion.
//
// Sec. 2.5, time stepping: particles advance with second-order leapfrog in its
// kick-drift-kick form with one global step per simulation; the step is eta
// times the smallest, over the cells, of the velocity dispersion of a cell
// over the largest acceleration in it.  Sec. 3.1: singlestep kicks, drifts and
// moves particles to their new cells (here: build_cells again) before the next
// force evaluation.
//
// Storage: positions, velocities and accelerations are FP32 in input order.
// A kick v + a dt and a drift x + v dt are evaluated in FP64 from the stored
// values, without contraction (the product rounded, then the sum), and rounded
// once to FP32; a drifted coordinate y is wrapped as y - L floor(y / L) and
// stored as 0 if its FP32 rounding reaches L.  Both kernels stream the arrays
// once (HBM-bound, 36 bytes per particle each).
//
// Timestep: per cell, with v_ref the velocity of the cell's first particle and
// d = v - v_ref, the sums S1 = sum d, S2 = sum |d|^2 and A = max |a|^2 give
// sigma^2 = S2 / n - |S1 / n|^2 (the shift keeps the difference well
// conditioned when the cell moves in bulk).  Cells with fewer than two
// particles or A = 0 do not constrain the step.  The work is cut by slot: one
// wave per kTsUnit sorted slots issues all of its loads at once, forms the
// sums per cell segment with a segmented scan across each batch of 64 slots,
// carries an open segment into the next batch, and at a cell's end either
// folds sigma/|a|max into a per-box minimum (atomic min on the bits of a
// non-negative double, so exact and order-free) or, for a cell that crosses a
// unit boundary, writes the unit's head or tail partial for k_ts_combine.  A
// comes either from the accelerations (gathered through the permutation) or,
// without them, from the per-cell maxima the force pass recorded.
//
// Merge (Table "tbl:timing": particles are stored cell by cell): the caller's
// per-particle arrays can be gathered into the sorted order of the last build,
// after which the handle's permutation is the identity; later passes then read
// and write those arrays nearly sequentially.
#include "nf_internal.h"

namespace anf {

namespace {

constexpr int kDtChunk = 24;
constexpr int kTsUnit = 256;                 // slots per wave of the timestep pass
constexpr int kTsBatches = kTsUnit / 64;
constexpr int kTsVals = 5;   // S1x, S1y, S1z, S2, A
// Per-box minima are kept in kTsSlots slots per box (a wave or boundary folds into slot index mod kTsSlots),
// so that the atomic minima of thousands of waves do not all meet on one address; a last kernel takes the
// minimum over the slots of each box.
constexpr int kTsSlots = 64;

struct DtChunk {
    double v[kDtChunk];
    int first, count;
};

__global__ void k_set_doubles(DtChunk c, double *dst) {
    int i = threadIdx.x;
    if (i < c.count) dst[c.first + i] = c.v[i];
}

__global__ void k_fill_u64(unsigned long long *p, int64_t n, unsigned long long v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ __launch_bounds__(256) void k_kick(float *__restrict__ vel, const float *__restrict__ acc, int64_t n3,
                                              const BoxDev *__restrict__ boxes, int n_boxes,
                                              const double *__restrict__ dt) {
#pragma clang fp contract(off)
    const double dt0 = dt[0];
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n3; e += (int64_t)gridDim.x * blockDim.x) {
        const double h = n_boxes > 1 ? dt[box_of_particle(boxes, n_boxes, e / 3)] : dt0;
        const double prod = (double)acc[e] * h;
        vel[e] = (float)((double)vel[e] + prod);
    }
}

__global__ __launch_bounds__(256) void k_drift(float *__restrict__ pos, const float *__restrict__ vel, int64_t n3,
                                               const BoxDev *__restrict__ boxes, int n_boxes,
                                               const double *__restrict__ dt) {
#pragma clang fp contract(off)
    const double dt0 = dt[0], L0 = boxes[0].L;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n3; e += (int64_t)gridDim.x * blockDim.x) {
        double h = dt0, L = L0;
        if (n_boxes > 1) {
            const int b = box_of_particle(boxes, n_boxes, e / 3);
            h = dt[b];
            L = boxes[b].L;
        }
        const double prod = (double)vel[e] * h;
        double y = (double)pos[e] + prod;
        const double q = floor(y / L);
        const double wrap = L * q;
        y = y - wrap;
        float f = (float)y;
        if ((double)f >= L) f = 0.0f;
        pos[e] = f;
    }
}

// Merge: caller arrays gathered into the sorted order (dst[s] = src[perm[s]]), then copied back.
__global__ __launch_bounds__(256) void k_permute_f32x3(const float *__restrict__ src, float *__restrict__ dst,
                                                       const int32_t *__restrict__ perm, int64_t n3) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n3; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t s = e / 3;
        dst[e] = src[3 * (int64_t)perm[s] + (e - 3 * s)];
    }
}

__global__ __launch_bounds__(256) void k_permute_i64(const int64_t *__restrict__ src, int64_t *__restrict__ dst,
                                                     const int32_t *__restrict__ perm, int64_t n) {
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < n; s += (int64_t)gridDim.x * blockDim.x)
        dst[s] = src[perm[s]];
}

__global__ __launch_bounds__(256) void k_iota_i32(int32_t *__restrict__ p, int64_t n) {
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < n; s += (int64_t)gridDim.x * blockDim.x)
        p[s] = (int32_t)s;
}

struct TsArgs {
    const float *vel;
    const float *acc;                    // accelerations, or nullptr: per-cell maxima of the force pass
    const unsigned long long *amax;      // [n_cells] bits of max |a|^2 per cell (used when acc is nullptr)
    const int32_t *keys;
    const int32_t *perm;
    const int32_t *cs;
    const BoxDev *boxes;
    int n_boxes;
    int64_t n;
    double *partials;             // [2 per unit][kTsVals]: head, tail
    unsigned long long *dmin;     // [n_boxes][kTsSlots] bits of the smallest sigma / |a|max, then [n_boxes] final
};

// |x|^2 with every product and sum rounded on its own, in a fixed order (the same value the caller gets
// from (x*x + y*y) + z*z in FP64).
__device__ inline double norm2(double x, double y, double z) {
#pragma clang fp contract(off)
    return x * x + y * y + z * z;
}

__device__ inline double cell_ratio(const double *t, int n, double A) {
    // sigma / |a|max, or a negative value when the cell does not constrain the step
    if (n < 2 || !(A > 0.0)) return -1.0;
    const double inv = 1.0 / n;
    const double m2 = (t[0] * t[0] + t[1] * t[1] + t[2] * t[2]) * inv * inv;
    double s2 = t[3] * inv - m2;
    s2 = s2 > 0.0 ? s2 : 0.0;
    return sqrt(s2) / sqrt(A);
}

__device__ inline void fold_min(unsigned long long *dmin, int box, int64_t slot, double r) {
    atomicMin(dmin + (int64_t)box * kTsSlots + slot % kTsSlots, (unsigned long long)__double_as_longlong(r));
}

// Three consecutive floats, read with one 12-byte load.
struct F3 {
    float x, y, z;
};

// One wave per unit of kTsUnit sorted slots.  Every load of the unit is issued before the first sum: keys
// and permutation entries (coalesced), then the velocities (and accelerations) gathered through the
// permutation.  The unit is reduced in batches of 64 slots.  The shift of a cell is the velocity of its
// first particle: a lane takes it from the lane where its cell starts in the batch, or from the segment
// still open at the end of the previous batch, or, for a cell that began before the unit, from one
// wave-uniform lookup.
template <bool FUSED>
__global__ __launch_bounds__(256) void k_ts_units(TsArgs a) {
    constexpr int NV = FUSED ? 4 : kTsVals;   // components of the scan (A comes from the force pass)
    const int lane = threadIdx.x & 63;
    const int64_t n_units = (a.n + kTsUnit - 1) / kTsUnit;
    const int64_t u = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (u >= n_units) return;
    const int64_t s0 = u * kTsUnit;
    const int64_t s1 = s0 + kTsUnit < a.n ? s0 + kTsUnit : a.n;
    int key[kTsBatches];
    float v[kTsBatches][3], g[kTsBatches][3];
#pragma unroll
    for (int b = 0; b < kTsBatches; b++) {
        const int64_t s = s0 + 64 * b + lane;
        key[b] = s < s1 ? a.keys[s] : -2;
        const int64_t p = s < s1 ? a.perm[s] : 0;
        F3 tv = {0.f, 0.f, 0.f}, tg = {0.f, 0.f, 0.f};
        if (s < s1) {
            tv = reinterpret_cast<const F3 *>(a.vel)[p];
            if (!FUSED) tg = reinterpret_cast<const F3 *>(a.acc)[p];
        }
        v[b][0] = tv.x;
        v[b][1] = tv.y;
        v[b][2] = tv.z;
        g[b][0] = tg.x;
        g[b][1] = tg.y;
        g[b][2] = tg.z;
    }
    const int unit_prev = s0 > 0 ? a.keys[s0 - 1] : -1;
    const int after = s1 < a.n ? a.keys[s1] : -1;
    float carry_ref[3] = {0.f, 0.f, 0.f};
    {
        const int k0 = __builtin_amdgcn_readfirstlane(key[0]);
        if (k0 == unit_prev) {   // the unit starts inside a cell: its first particle lies before the unit
            const int64_t pf = a.perm[a.cs[k0]];
#pragma unroll
            for (int d = 0; d < 3; d++) carry_ref[d] = a.vel[3 * pf + d];
        }
    }
    double carry[kTsVals] = {0.0, 0.0, 0.0, 0.0, 0.0};
    int carry_key = -1;
    int lane_box = -1;
    double lane_min = 0.0;
#pragma unroll
    for (int b = 0; b < kTsBatches; b++) {
        const int64_t b0 = s0 + 64 * b;
        if (b0 >= s1) break;
        const int nb = (int)(s1 - b0 < 64 ? s1 - b0 : 64);
        const bool live = lane < nb;
        const int k = key[b];
        const int up = __shfl_up(k, 1);
        const int before = b == 0 ? unit_prev : __shfl(key[b > 0 ? b - 1 : 0], 63);
        const bool start = live && k != (lane == 0 ? before : up);   // the first slot of its cell
        const unsigned long long startmask = __ballot(start);
        const unsigned long long below = startmask & (lane == 63 ? ~0ull : ((2ull << lane) - 1));
        const int sl = below ? 63 - __builtin_clzll(below) : 0;
        float r[3];
#pragma unroll
        for (int d = 0; d < 3; d++) {
            const float t = __shfl(v[b][d], sl);
            r[d] = below ? t : carry_ref[d];
        }
        // the cell of the next batch's first slot (every lane takes part in the cross-lane read)
        const int first_next = __shfl(key[b + 1 < kTsBatches ? b + 1 : b], 0);
        int nxt = __shfl_down(k, 1);
        if (lane == nb - 1) nxt = (b0 + 64 < s1) ? first_next : ~k;   // the unit's end closes a segment
        const bool end = live && k != nxt;
        const unsigned long long endmask = __ballot(end);
        double x[kTsVals] = {0.0, 0.0, 0.0, 0.0, 0.0};
        if (live) {
            const double dx = (double)v[b][0] - (double)r[0];
            const double dy = (double)v[b][1] - (double)r[1];
            const double dz = (double)v[b][2] - (double)r[2];
            x[0] = dx;
            x[1] = dy;
            x[2] = dz;
            x[3] = norm2(dx, dy, dz);
            if (!FUSED) x[4] = norm2((double)g[b][0], (double)g[b][1], (double)g[b][2]);
        }
        // segmented inclusive scan over the lanes of the batch (sums, and a max for A)
        bool f = lane == 0 || k != up;
        for (int off = 1; off < 64; off <<= 1) {
            double y[kTsVals];
#pragma unroll
            for (int q = 0; q < NV; q++) y[q] = __shfl_up(x[q], off);
            const bool fy = __shfl_up((int)f, off) != 0;
            if (lane >= off) {
                if (!f) {
#pragma unroll
                    for (int q = 0; q < 4; q++) x[q] += y[q];
                    if (!FUSED) x[4] = x[4] > y[4] ? x[4] : y[4];
                }
                f = f || fy;
            }
        }
        const int c0 = __builtin_amdgcn_readfirstlane(k);
        const bool add_carry = carry_key >= 0 && c0 == carry_key;
        const int e0 = endmask ? __builtin_ctzll(endmask) : -1;
        if (end) {
            if (lane == e0 && add_carry) {
#pragma unroll
                for (int q = 0; q < 4; q++) x[q] += carry[q];
                if (!FUSED) x[4] = x[4] > carry[4] ? x[4] : carry[4];
            }
            const bool started = k != unit_prev;
            const bool ends = (b0 + lane + 1 < s1) || after != k;
            if (started && ends) {
                const double A = FUSED ? __longlong_as_double((long long)a.amax[k]) : x[4];
                const double rr = cell_ratio(x, a.cs[k + 1] - a.cs[k], A);
                if (rr >= 0.0) {
                    const int bx = a.n_boxes > 1 ? box_of_cell(a.boxes, a.n_boxes, k) : 0;
                    if (bx != lane_box) {
                        if (lane_box >= 0) fold_min(a.dmin, lane_box, u, lane_min);
                        lane_box = bx;
                        lane_min = rr;
                    } else {
                        lane_min = rr < lane_min ? rr : lane_min;
                    }
                }
            } else {
                double *o = a.partials + (2 * u + (started ? 1 : 0)) * kTsVals;
#pragma unroll
                for (int q = 0; q < kTsVals; q++) o[q] = x[q];
            }
        }
        // the segment still open at the batch's end becomes the carry (with its shift)
        if (!((endmask >> (nb - 1)) & 1)) {
            double t[kTsVals];
#pragma unroll
            for (int q = 0; q < kTsVals; q++) t[q] = __shfl(x[q], nb - 1);
            if (endmask == 0 && add_carry) {
#pragma unroll
                for (int q = 0; q < 4; q++) t[q] += carry[q];
                t[4] = t[4] > carry[4] ? t[4] : carry[4];
            }
#pragma unroll
            for (int q = 0; q < kTsVals; q++) carry[q] = t[q];
            carry_key = __shfl(k, nb - 1);
#pragma unroll
            for (int d = 0; d < 3; d++) carry_ref[d] = __shfl(r[d], nb - 1);
        } else {
            carry_key = -1;
        }
    }
    // the wave's minima, one atomic per box present in the wave (normally one box)
    for (;;) {
        const unsigned long long pending = __ballot(lane_box >= 0);
        if (!pending) break;
        const int bx = __shfl(lane_box, __builtin_ctzll(pending));
        double m = lane_box == bx ? lane_min : __longlong_as_double(0x7FF0000000000000ll);
        for (int off = 32; off > 0; off >>= 1) {
            const double y = __shfl_xor(m, off);
            m = y < m ? y : m;
        }
        if (lane == 0) fold_min(a.dmin, bx, u, m);
        if (lane_box == bx) lane_box = -1;
    }
}

// Cells that cross unit boundaries, one wave per boundary: at the first boundary a cell crosses, the
// lanes add the head partials of the units it continues into (lane l takes units u + l, u + l + 64, ...),
// a fixed butterfly combines the lanes, and lane 0 adds the tail partial of the unit where the cell begins.
// Fixed orders throughout, so the result does not depend on scheduling.
template <bool FUSED>
__global__ __launch_bounds__(256) void k_ts_combine(TsArgs a) {
    const int lane = threadIdx.x & 63;
    const int64_t n_units = (a.n + kTsUnit - 1) / kTsUnit;
    const int64_t u = 1 + (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (u >= n_units) return;
    const int c = a.keys[u * kTsUnit];
    if (a.keys[u * kTsUnit - 1] != c) return;
    if (u >= 2 && a.keys[(u - 1) * kTsUnit - 1] == c) return;
    const int64_t last = (a.cs[c + 1] - 1) / kTsUnit;   // unit of the cell's last slot
    double t[kTsVals] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int64_t w = u + lane; w <= last; w += 64) {
        const double *h = a.partials + (2 * w) * kTsVals;
#pragma unroll
        for (int q = 0; q < 4; q++) t[q] += h[q];
        if (!FUSED) t[4] = t[4] > h[4] ? t[4] : h[4];
    }
    for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
        for (int q = 0; q < 4; q++) t[q] += __shfl_xor(t[q], off);
        if (!FUSED) {
            const double y = __shfl_xor(t[4], off);
            t[4] = t[4] > y ? t[4] : y;
        }
    }
    if (lane != 0) return;
    const double *tail = a.partials + (2 * (u - 1) + 1) * kTsVals;
    double s[kTsVals];
#pragma unroll
    for (int q = 0; q < 4; q++) s[q] = tail[q] + t[q];
    const double A = FUSED ? __longlong_as_double((long long)a.amax[c]) : (tail[4] > t[4] ? tail[4] : t[4]);
    const double r = cell_ratio(s, a.cs[c + 1] - a.cs[c], A);
    if (r >= 0.0) fold_min(a.dmin, a.n_boxes > 1 ? box_of_cell(a.boxes, a.n_boxes, c) : 0, u, r);
}

// Minimum over the slots of each box, into the final words after the slots.
__global__ void k_ts_final(unsigned long long *dmin, int n_boxes) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n_boxes) return;
    unsigned long long m = dmin[(int64_t)b * kTsSlots];
    for (int q = 1; q < kTsSlots; q++) {
        const unsigned long long y = dmin[(int64_t)b * kTsSlots + q];
        m = y < m ? y : m;
    }
    dmin[(int64_t)n_boxes * kTsSlots + b] = m;
}

int grid_of(int64_t n, int threads, int device, int per_cu) {
    int cus = 1;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || cus < 1) cus = 1;
    const int64_t want = (n + threads - 1) / threads;
    const int64_t cap = (int64_t)cus * per_cu;
    return (int)(want < cap ? (want > 0 ? want : 1) : cap);
}

}  // namespace

hipError_t upload_box_doubles(const double *host, int n_boxes, double *dev, hipStream_t st) {
    for (int first = 0; first < n_boxes; first += kDtChunk) {
        DtChunk ch;
        ch.first = first;
        ch.count = n_boxes - first < kDtChunk ? n_boxes - first : kDtChunk;
        for (int k = 0; k < kDtChunk; k++) ch.v[k] = k < ch.count ? host[first + k] : 0.0;
        hipLaunchKernelGGL(k_set_doubles, dim3(1), dim3(kDtChunk), 0, st, ch, dev);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_kick(float *vel, const float *acc, int64_t n, const BoxDev *boxes, int n_boxes, const double *dt,
                       int device, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_kick, dim3(grid_of(3 * n, 256, device, 32)), dim3(256), 0, st, vel, acc, 3 * n, boxes,
                       n_boxes, dt);
    return hipGetLastError();
}

hipError_t launch_drift(float *pos, const float *vel, int64_t n, const BoxDev *boxes, int n_boxes, const double *dt,
                        int device, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_drift, dim3(grid_of(3 * n, 256, device, 32)), dim3(256), 0, st, pos, vel, 3 * n, boxes,
                       n_boxes, dt);
    return hipGetLastError();
}

hipError_t launch_reorder(float *const *vec3, int n_vec3, int64_t *ids, int32_t *perm, int64_t n, void *scratch,
                          int device, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const unsigned g3 = (unsigned)grid_of(3 * n, 256, device, 32), g1 = (unsigned)grid_of(n, 256, device, 32);
    hipError_t e;
    for (int k = 0; k < n_vec3; k++) {
        float *tmp = (float *)scratch;
        hipLaunchKernelGGL(k_permute_f32x3, dim3(g3), dim3(256), 0, st, vec3[k], tmp, perm, 3 * n);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if ((e = hipMemcpyAsync(vec3[k], tmp, (size_t)n * 12, hipMemcpyDeviceToDevice, st)) != hipSuccess) return e;
    }
    if (ids) {
        int64_t *tmp = (int64_t *)scratch;
        hipLaunchKernelGGL(k_permute_i64, dim3(g1), dim3(256), 0, st, ids, tmp, perm, n);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if ((e = hipMemcpyAsync(ids, tmp, (size_t)n * 8, hipMemcpyDeviceToDevice, st)) != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_iota_i32, dim3(g1), dim3(256), 0, st, perm, n);
    return hipGetLastError();
}

size_t timestep_partial_doubles(int64_t n) {
    const int64_t units = (n + kTsUnit - 1) / kTsUnit;
    return (size_t)(2 * (units > 0 ? units : 1)) * kTsVals;
}

hipError_t launch_fill_u64(unsigned long long *p, int64_t n, unsigned long long v, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const int64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(k_fill_u64, dim3((unsigned)(blocks < 65536 ? blocks : 65536)), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}

hipError_t launch_timestep(const float *vel, const float *acc, const unsigned long long *amax, const int32_t *keys,
                           const int32_t *perm, const int32_t *cs, const BoxDev *boxes, int n_boxes, int64_t n,
                           double *partials, unsigned long long *dmin, hipStream_t st) {
    const unsigned long long inf_bits = 0x7FF0000000000000ull;
    const int64_t nslots = (int64_t)n_boxes * kTsSlots;
    hipError_t e = launch_fill_u64(dmin, nslots, inf_bits, st);
    if (e != hipSuccess) return e;
    auto final_min = [&]() {
        hipLaunchKernelGGL(k_ts_final, dim3((unsigned)((n_boxes + 63) / 64)), dim3(64), 0, st, dmin, n_boxes);
        return hipGetLastError();
    };
    if (n <= 0) return final_min();
    TsArgs a;
    a.vel = vel;
    a.acc = acc;
    a.amax = amax;
    a.keys = keys;
    a.perm = perm;
    a.cs = cs;
    a.boxes = boxes;
    a.n_boxes = n_boxes;
    a.n = n;
    a.partials = partials;
    a.dmin = dmin;
    const int64_t n_units = (n + kTsUnit - 1) / kTsUnit;
    const bool fused = acc == nullptr;
    hipLaunchKernelGGL(fused ? k_ts_units<true> : k_ts_units<false>, dim3((unsigned)((n_units + 3) / 4)), dim3(256),
                       0, st, a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (n_units >= 2) {
        hipLaunchKernelGGL(fused ? k_ts_combine<true> : k_ts_combine<false>,
                           dim3((unsigned)((n_units - 1 + 3) / 4)), dim3(256), 0, st, a);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return final_min();
}

size_t timestep_min_words(int n_boxes) { return (size_t)n_boxes * (kTsSlots + 1); }

size_t timestep_min_offset(int n_boxes) { return (size_t)n_boxes * kTsSlots; }

}  // namespace anf

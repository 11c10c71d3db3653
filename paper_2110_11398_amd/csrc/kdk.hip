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
// Timestep: per cell, with v_ref the velocity of the cell's first particle (gathered
// once per cell by k_ts_ref) and
// d = v - v_ref, the sums S1 = sum d, S2 = sum |d|^2 and A = max |a|^2 give
// sigma^2 = S2 / n - |S1 / n|^2 (the shift keeps the difference well
// conditioned when the cell moves in bulk).  Cells with fewer than two
// particles or A = 0 do not constrain the step.  The work is cut by slot like
// the multipoles: a wave walks kTsUnit sorted slots 64 at a time, forms the five
// sums per cell segment with a segmented scan across the wave, carries an open
// segment into the next batch, and at a cell's end either folds sigma/|a|max
// into a per-box minimum (atomic min on the bits of a non-negative double, so
// exact and order-free) or, for a cell that crosses a unit boundary, writes the
// unit's head or tail partial for k_ts_combine.
//
// Merge (Table "tbl:timing": particles are stored cell by cell): the caller's
// per-particle arrays can be gathered into the sorted order of the last build,
// after which the handle's permutation is the identity; later passes then read
// and write those arrays nearly sequentially.
#include "nf_internal.h"

namespace anf {

namespace {

constexpr int kDtChunk = 24;
constexpr int kTsUnit = 1024;
constexpr int kTsVals = 5;   // S1x, S1y, S1z, S2, A

struct DtChunk {
    double v[kDtChunk];
    int first, count;
};

__global__ void k_set_doubles(DtChunk c, double *dst) {
    int i = threadIdx.x;
    if (i < c.count) dst[c.first + i] = c.v[i];
}

__global__ void k_fill_u64(unsigned long long *p, int64_t n, unsigned long long v) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
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
    const float *acc;
    const int32_t *keys;
    const int32_t *perm;
    const int32_t *cs;
    const BoxDev *boxes;
    int n_boxes;
    int64_t n;
    double *partials;             // [2 per unit][kTsVals]: head, tail
    unsigned long long *dmin;     // [n_boxes] bits of the smallest sigma / |a|max
    const float *ref;             // [n_cells][3] velocity of each occupied cell's first particle
};

// Reference velocity of every occupied cell: the velocity of its first sorted particle (read once per cell,
// so the per-particle pass below has no chain of dependent lookups for it).
__global__ __launch_bounds__(256) void k_ts_ref(const float *__restrict__ vel, const int32_t *__restrict__ perm,
                                                const int32_t *__restrict__ cs, int64_t n_cells,
                                                float *__restrict__ ref) {
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n_cells;
         c += (int64_t)gridDim.x * blockDim.x) {
        const int s0 = cs[c];
        if (cs[c + 1] > s0) {
            const int64_t r = perm[s0];
            ref[3 * c + 0] = vel[3 * r + 0];
            ref[3 * c + 1] = vel[3 * r + 1];
            ref[3 * c + 2] = vel[3 * r + 2];
        }
    }
}

__device__ inline double cell_ratio(const double *t, int n) {
    // sigma / |a|max, or a negative value when the cell does not constrain the step
    if (n < 2 || !(t[4] > 0.0)) return -1.0;
    const double inv = 1.0 / n;
    const double m2 = (t[0] * t[0] + t[1] * t[1] + t[2] * t[2]) * inv * inv;
    double s2 = t[3] * inv - m2;
    s2 = s2 > 0.0 ? s2 : 0.0;
    return sqrt(s2) / sqrt(t[4]);
}

__device__ inline void fold_min(unsigned long long *dmin, int box, double r) {
    atomicMin(dmin + box, (unsigned long long)__double_as_longlong(r));
}

__global__ __launch_bounds__(64) void k_ts_units(TsArgs a) {
    const int lane = threadIdx.x;
    const int64_t n_units = (a.n + kTsUnit - 1) / kTsUnit;
    const unsigned G = gridDim.x;
    const unsigned per_xcd = G / kQueues;
    const unsigned vb = (blockIdx.x % kQueues) * per_xcd + blockIdx.x / kQueues;
    const int64_t chunk = (n_units + G - 1) / G;
    const int64_t u_begin = (int64_t)vb * chunk;
    const int64_t u_end = u_begin + chunk < n_units ? u_begin + chunk : n_units;
    int lane_box = -1;
    double lane_min = 0.0;
    for (int64_t u = u_begin; u < u_end; u++) {
        const int64_t s0 = u * kTsUnit;
        const int64_t s1 = s0 + kTsUnit < a.n ? s0 + kTsUnit : a.n;
        const int unit_prev = s0 > 0 ? a.keys[s0 - 1] : -1;
        const int after = s1 < a.n ? a.keys[s1] : -1;
        double carry[kTsVals] = {0.0, 0.0, 0.0, 0.0, 0.0};
        int carry_key = -1;
        // two-deep pipeline: while a batch is reduced, the velocities, accelerations and reference velocities
        // of the next batch are in flight (gathered through the permutation), and the keys and permutation
        // entries of the batch after it
        int key_n = s0 + lane < s1 ? a.keys[s0 + lane] : -2;
        int perm_n = s0 + lane < s1 ? a.perm[s0 + lane] : 0;
        float v_n[3] = {0.f, 0.f, 0.f}, g_n[3] = {0.f, 0.f, 0.f}, r_n[3] = {0.f, 0.f, 0.f};
        if (s0 + lane < s1) {
            const float *vr = a.ref + 3 * (int64_t)key_n;
#pragma unroll
            for (int d = 0; d < 3; d++) {
                v_n[d] = a.vel[3 * (int64_t)perm_n + d];
                g_n[d] = a.acc[3 * (int64_t)perm_n + d];
                r_n[d] = vr[d];
            }
        }
        int key_nn = s0 + 64 + lane < s1 ? a.keys[s0 + 64 + lane] : -2;
        int perm_nn = s0 + 64 + lane < s1 ? a.perm[s0 + 64 + lane] : 0;
        for (int64_t b0 = s0; b0 < s1; b0 += 64) {
            const int nb = (int)(s1 - b0 < 64 ? s1 - b0 : 64);
            const bool live = lane < nb;
            const int key = key_n;
            float v[3], g[3], r[3];
#pragma unroll
            for (int d = 0; d < 3; d++) {
                v[d] = v_n[d];
                g[d] = g_n[d];
                r[d] = r_n[d];
            }
            const int64_t b1 = b0 + 64, b2 = b0 + 128;
            const bool live_n = b1 + lane < s1;
            key_n = key_nn;
            perm_n = perm_nn;
            if (live_n) {
                const float *vr = a.ref + 3 * (int64_t)key_n;
#pragma unroll
                for (int d = 0; d < 3; d++) {
                    v_n[d] = a.vel[3 * (int64_t)perm_n + d];
                    g_n[d] = a.acc[3 * (int64_t)perm_n + d];
                    r_n[d] = vr[d];
                }
            }
            key_nn = b2 + lane < s1 ? a.keys[b2 + lane] : -2;
            perm_nn = b2 + lane < s1 ? a.perm[b2 + lane] : 0;
            const int first_next = __builtin_amdgcn_readfirstlane(key_n);   // cell of slot b1 when b1 < s1
            const int prevk = __shfl_up(key, 1);
            int nxt = __shfl_down(key, 1);
            if (lane == nb - 1) nxt = (b1 < s1) ? first_next : ~key;       // the unit's end closes a segment
            const bool end = live && key != nxt;
            const uint64_t endmask = __ballot(end);
            double x[kTsVals] = {0.0, 0.0, 0.0, 0.0, 0.0};
            if (live) {
                const double dx = (double)v[0] - (double)r[0];
                const double dy = (double)v[1] - (double)r[1];
                const double dz = (double)v[2] - (double)r[2];
                const double ax = g[0], ay = g[1], az = g[2];
                x[0] = dx;
                x[1] = dy;
                x[2] = dz;
                x[3] = dx * dx + dy * dy + dz * dz;
                x[4] = ax * ax + ay * ay + az * az;
            }
            // segmented inclusive scan over the lanes (sums, and a max for A)
            bool f = lane == 0 || key != prevk;
            for (int off = 1; off < 64; off <<= 1) {
                double y[kTsVals];
#pragma unroll
                for (int k = 0; k < kTsVals; k++) y[k] = __shfl_up(x[k], off);
                const bool fy = __shfl_up((int)f, off) != 0;
                if (lane >= off) {
                    if (!f) {
#pragma unroll
                        for (int k = 0; k < 4; k++) x[k] += y[k];
                        x[4] = x[4] > y[4] ? x[4] : y[4];
                    }
                    f = f || fy;
                }
            }
            const int c0 = __builtin_amdgcn_readfirstlane(key);
            const bool add_carry = carry_key >= 0 && c0 == carry_key;
            const int e0 = endmask ? __builtin_ctzll(endmask) : -1;
            if (end) {
                if (lane == e0 && add_carry) {
#pragma unroll
                    for (int k = 0; k < 4; k++) x[k] += carry[k];
                    x[4] = x[4] > carry[4] ? x[4] : carry[4];
                }
                const bool started = key != unit_prev;
                const bool ends = (b0 + lane + 1 < s1) || after != key;
                if (started && ends) {
                    const double r = cell_ratio(x, a.cs[key + 1] - a.cs[key]);
                    if (r >= 0.0) {
                        const int bx = a.n_boxes > 1 ? box_of_cell(a.boxes, a.n_boxes, key) : 0;
                        if (bx != lane_box) {
                            if (lane_box >= 0) fold_min(a.dmin, lane_box, lane_min);
                            lane_box = bx;
                            lane_min = r;
                        } else {
                            lane_min = r < lane_min ? r : lane_min;
                        }
                    }
                } else {
                    double *o = a.partials + (2 * u + (started ? 1 : 0)) * kTsVals;
#pragma unroll
                    for (int k = 0; k < kTsVals; k++) o[k] = x[k];
                }
            }
            // the segment still open at the batch's end becomes the carry
            if (!((endmask >> (nb - 1)) & 1)) {
                double t[kTsVals];
#pragma unroll
                for (int k = 0; k < kTsVals; k++) t[k] = __shfl(x[k], nb - 1);
                if (endmask == 0 && add_carry) {
#pragma unroll
                    for (int k = 0; k < 4; k++) t[k] += carry[k];
                    t[4] = t[4] > carry[4] ? t[4] : carry[4];
                }
#pragma unroll
                for (int k = 0; k < kTsVals; k++) carry[k] = t[k];
                carry_key = __shfl(key, nb - 1);
            } else {
                carry_key = -1;
            }
        }
    }
    if (lane_box >= 0) fold_min(a.dmin, lane_box, lane_min);
}

// Cells that cross unit boundaries: the tail partial of the unit where the cell begins and the head
// partials of the units it continues into (sums added, maxima taken), then the ratio.
__global__ __launch_bounds__(64) void k_ts_combine(TsArgs a) {
    const int64_t n_units = (a.n + kTsUnit - 1) / kTsUnit;
    for (int64_t u = 1 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n_units;
         u += (int64_t)gridDim.x * blockDim.x) {
        const int c = a.keys[u * kTsUnit];
        if (a.keys[u * kTsUnit - 1] != c) continue;
        if (u >= 2 && a.keys[(u - 1) * kTsUnit - 1] == c) continue;
        double t[kTsVals];
#pragma unroll
        for (int k = 0; k < kTsVals; k++) t[k] = a.partials[(2 * (u - 1) + 1) * kTsVals + k];
        const int64_t last = (a.cs[c + 1] - 1) / kTsUnit;   // unit of the cell's last slot
        for (int64_t v = u; v <= last; v++) {
            const double *h = a.partials + (2 * v) * kTsVals;
#pragma unroll
            for (int k = 0; k < 4; k++) t[k] += h[k];
            t[4] = t[4] > h[4] ? t[4] : h[4];
        }
        const double r = cell_ratio(t, a.cs[c + 1] - a.cs[c]);
        if (r >= 0.0) fold_min(a.dmin, a.n_boxes > 1 ? box_of_cell(a.boxes, a.n_boxes, c) : 0, r);
    }
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

hipError_t launch_timestep(const float *vel, const float *acc, const int32_t *keys, const int32_t *perm,
                           const int32_t *cs, const BoxDev *boxes, int n_boxes, int64_t n, int64_t n_cells,
                           double *partials, float *ref, unsigned long long *dmin, int device, hipStream_t st) {
    const unsigned long long inf_bits = 0x7FF0000000000000ull;
    hipLaunchKernelGGL(k_fill_u64, dim3((unsigned)((n_boxes + 255) / 256)), dim3(256), 0, st, dmin,
                       (int64_t)n_boxes, inf_bits);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || n <= 0) return e;
    TsArgs a;
    a.vel = vel;
    a.acc = acc;
    a.keys = keys;
    a.perm = perm;
    a.cs = cs;
    a.boxes = boxes;
    a.n_boxes = n_boxes;
    a.n = n;
    a.partials = partials;
    a.dmin = dmin;
    a.ref = ref;
    hipLaunchKernelGGL(k_ts_ref, dim3((unsigned)grid_of(n_cells, 256, device, 32)), dim3(256), 0, st, vel, perm, cs,
                       n_cells, ref);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    int cus = 1;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || cus < 1) cus = 1;
    const int64_t n_units = (n + kTsUnit - 1) / kTsUnit;
    int64_t grid = std::min<int64_t>(n_units, (int64_t)cus * 32);
    grid = (grid + kQueues - 1) / kQueues * kQueues;
    hipLaunchKernelGGL(k_ts_units, dim3((unsigned)grid), dim3(64), 0, st, a);
    if ((e = hipGetLastError()) != hipSuccess || n_units < 2) return e;
    const int64_t cgrid = std::min<int64_t>((n_units + 63) / 64, (int64_t)cus * 4);
    hipLaunchKernelGGL(k_ts_combine, dim3((unsigned)cgrid), dim3(64), 0, st, a);
    return hipGetLastError();
}

}  // namespace anf

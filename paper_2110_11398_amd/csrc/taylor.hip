// Far-field force from per-cell Taylor series, co-added to the near field.
//
// Sec. 3.1: the far-field acceleration is a Taylor expansion, to order p, of
// the potential about each cell centre; singlestep evaluates its gradient at
// every particle and adds it to the near-field force ("Taylor Force", Table
// "tbl:timing").  With (u, v, w) the particle's position relative to its cell
// centre in cell widths (the layout build_cells produced) and
//     Phi = sum_{a+b+k <= p} T^(a,b,k) u^a v^b w^k,
// the far field is -grad_x Phi = -(K/L) grad_u Phi, added to acc.
//
// Work is cut by particle, not by cell: a wave owns a contiguous run of slots
// of the cell-sorted layout, so every wave carries the same work whatever the
// occupancy of the cells (a halo core spans many waves, a sparse region packs
// several cells into one).  It walks the run in steps of up to 64 slots that
// cover at most kCells cells, whose coefficients are staged in LDS; each lane
// reads its own cell's block.  Waves on one XCD take adjacent runs, so a cell
// whose particles straddle two runs is read from that XCD's L2.
//
// Per particle: for every column (b, k) the polynomial P_bk(u) =
// sum_a T^(a,b,k) u^a and its derivative come from one Horner pass, then
//     d/du Phi = sum P'_bk v^b w^k,  d/dv Phi = sum P_bk b v^(b-1) w^k,
//     d/dw Phi = sum P_bk v^b k w^(k-1),
// all in FP64 with the order p a compile-time constant, so every power stays
// in registers.
#include "nf_internal.h"

namespace anf {

namespace {

constexpr int kTyMaxOrder = 10;
// LDS per wave for staged coefficients: 6 KB (4 cells of order 8 per step of 64 slots), or 16 KB (12 cells)
// where cells hold fewer than 16 particles on average.  Measured at order 8: clustered workload (64 per cell)
// 4 / 6 / 8 / 16 KB: 0.548 / 0.534 / 0.60 / 0.77 ms; late-time workload (8 per cell) 8 / 16 KB: 10.24 / 8.39 ms
constexpr int kTyStageBytes = 6144, kTyStageBytesSparse = 16384;

// Position of component (a, b, k) in the degree / a-descending / b-descending order.
__host__ __device__ constexpr int comp_index(int a, int b, int k) {
    const int n = a + b + k;
    return n * (n + 1) * (n + 2) / 6 + (n - a) * (n - a + 1) / 2 + (n - a - b);
}

struct TyArgs {
    const float4 *spos;
    const int32_t *keys;   // cell of every slot (sorted)
    const int32_t *perm;   // input index of every slot
    const BoxDev *boxes;
    int n_boxes;
    int64_t n;             // particles (slots)
    const double *taylor;
    float *acc;
};

__device__ inline void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// -grad_(u,v,w) of the order-P series with coefficients T at (u, v, w), added to (gx, gy, gz) with the sign
// of +grad (the caller subtracts).
template <int P>
__device__ __forceinline__ void taylor_gradient(const double *__restrict__ T, double u, double v, double w,
                                                double &gx, double &gy, double &gz) {
    double pv[P + 1], pw[P + 1];
    pv[0] = pw[0] = 1.0;
#pragma unroll
    for (int q = 1; q <= P; q++) {
        pv[q] = pv[q - 1] * v;
        pw[q] = pw[q - 1] * w;
    }
#pragma unroll
    for (int b = 0; b <= P; b++) {
#pragma unroll
        for (int k = 0; k + b <= P; k++) {
            // Horner over a = top..0 for the value and the derivative of P_bk(u)
            const int top = P - b - k;
            double val = T[comp_index(top, b, k)];
            double der = 0.0;
#pragma unroll
            for (int aa = top - 1; aa >= 0; aa--) {
                der = der * u + val;
                val = val * u + T[comp_index(aa, b, k)];
            }
            const double vw = pv[b] * pw[k];
            gx += der * vw;
            if (b > 0) gy += val * (b * pv[b - 1]) * pw[k];
            if (k > 0) gz += val * pv[b] * (k * pw[k - 1]);
            // keep each column's reads next to their use (no hoisting of all of them)
            __builtin_amdgcn_sched_barrier(0);
        }
    }
}

template <int P, int STAGE_BYTES>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(P >= 9 ? 2 : 4, 8))) void k_taylor(TyArgs a, const double *__restrict__ taylor) {
    constexpr int NC = (P + 1) * (P + 2) * (P + 3) / 6;
    constexpr int kCells = STAGE_BYTES / (NC * 8) > 0 ? STAGE_BYTES / (NC * 8) : 1;
    __shared__ double tc[kCells * NC];
    const int lane = threadIdx.x;
    // XCD-aware contiguous chunks of slots: block i runs on XCD i % 8; the blocks of one XCD take adjacent chunks
    const unsigned G = gridDim.x;
    const unsigned per_xcd = G / kQueues;
    const unsigned vb = (blockIdx.x % kQueues) * per_xcd + blockIdx.x / kQueues;
    const int64_t chunk = ((a.n + G - 1) / G + 63) / 64 * 64;
    const int64_t s_begin = (int64_t)vb * chunk;
    const int64_t s_end = s_begin + chunk < a.n ? s_begin + chunk : a.n;
    // Steps of up to 64 slots that cover at most kCells cells: every lane of a step evaluates with the
    // staged coefficients of its own cell, and the next step starts at the first slot not taken.  The walk is
    // software-pipelined: while a step is evaluated, the next step's coefficients, coordinates and
    // permutation entries are already in flight, and the keys of the step after it.
    constexpr int kIters = (kCells * NC + 63) / 64;
    if (s_begin >= s_end) return;
    const int kNone = 0x7fffffff;
    int64_t s = s_begin;
    int key = s + lane < s_end ? a.keys[s + lane] : kNone;
    // window of the current step
    int c_lo = __builtin_amdgcn_readfirstlane(key);                  // lane 0 is always in range
    bool live = key - c_lo < kCells;                                  // keys are sorted: a prefix of lanes
    int taken = __builtin_popcountll(__ballot(live));
    int c_hi = __builtin_amdgcn_readlane(key, taken - 1);
    double stage[kIters];
    {
        const int nv = (c_hi - c_lo + 1) * NC;
        const double *src = taylor + (int64_t)c_lo * NC;
#pragma unroll
        for (int it = 0; it < kIters; it++) stage[it] = lane + 64 * it < nv ? src[lane + 64 * it] : 0.0;
    }
    float4 sp = live ? a.spos[s + lane] : make_float4(0.f, 0.f, 0.f, 0.f);
    int pi = live ? a.perm[s + lane] : 0;
    int64_t s_next = s + taken;
    int key_next = s_next + lane < s_end ? a.keys[s_next + lane] : kNone;
    for (;;) {
        // the current step's coefficients to LDS
        const int nv = (c_hi - c_lo + 1) * NC;
        wave_sync();
#pragma unroll
        for (int it = 0; it < kIters; it++)
            if (lane + 64 * it < nv) tc[lane + 64 * it] = stage[it];
        wave_sync();
        // the next step: its window from the keys already loaded; issue its loads and the keys after it
        const bool more = s_next < s_end;
        int c_lo_n = 0, taken_n = 0, c_hi_n = 0, pi_n = 0, key_after = kNone;
        bool live_n = false;
        float4 sp_n = make_float4(0.f, 0.f, 0.f, 0.f);
        int64_t s_after = s_end;
        if (more) {
            c_lo_n = __builtin_amdgcn_readfirstlane(key_next);
            live_n = key_next - c_lo_n < kCells;
            taken_n = __builtin_popcountll(__ballot(live_n));
            c_hi_n = __builtin_amdgcn_readlane(key_next, taken_n - 1);
            const int nv_n = (c_hi_n - c_lo_n + 1) * NC;
            const double *src = taylor + (int64_t)c_lo_n * NC;
#pragma unroll
            for (int it = 0; it < kIters; it++) stage[it] = lane + 64 * it < nv_n ? src[lane + 64 * it] : 0.0;
            if (live_n) {
                sp_n = a.spos[s_next + lane];
                pi_n = a.perm[s_next + lane];
            }
            s_after = s_next + taken_n;
            key_after = s_after + lane < s_end ? a.keys[s_after + lane] : kNone;
        }
        // evaluate the current step
        if (live) {
            const double u = sp.x, v = sp.y, w = sp.z;
            const int bi = a.n_boxes > 1 ? box_of_cell(a.boxes, a.n_boxes, key) : 0;
            const double sc = a.boxes[bi].s;
            double gx = 0.0, gy = 0.0, gz = 0.0;
            taylor_gradient<P>(tc + (key - c_lo) * NC, u, v, w, gx, gy, gz);
            float *o = a.acc + 3 * (int64_t)pi;
            o[0] = (float)((double)o[0] - sc * gx);
            o[1] = (float)((double)o[1] - sc * gy);
            o[2] = (float)((double)o[2] - sc * gz);
        }
        if (!more) break;
        // rotate: the next step becomes the current one
        s = s_next;
        key = key_next;
        c_lo = c_lo_n;
        live = live_n;
        taken = taken_n;
        c_hi = c_hi_n;
        sp = sp_n;
        pi = pi_n;
        s_next = s_after;
        key_next = key_after;
    }
}

typedef void (*TyKernel)(TyArgs, const double *);

template <int P>
TyKernel pick_taylor(int p, bool sparse) {
    if constexpr (P > kTyMaxOrder) {
        return nullptr;
    } else {
        if (p == P) return sparse ? k_taylor<P, kTyStageBytesSparse> : k_taylor<P, kTyStageBytes>;
        return pick_taylor<P + 1>(p, sparse);
    }
}

}  // namespace

int taylor_max_order() { return kTyMaxOrder; }

hipError_t launch_taylor(const float4 *spos, const int32_t *keys, const int32_t *perm, const BoxDev *boxes,
                         int n_boxes, int64_t n, int64_t n_cells, int p, const double *taylor, float *acc,
                         int device, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    TyKernel kfn = pick_taylor<0>(p, n < 16 * n_cells);
    if (!kfn) return hipErrorInvalidValue;
    TyArgs a;
    a.spos = spos;
    a.keys = keys;
    a.perm = perm;
    a.boxes = boxes;
    a.n_boxes = n_boxes;
    a.n = n;
    a.taylor = taylor;
    a.acc = acc;
    int cus = 1;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || cus < 1) cus = 1;
    // a multiple of 8 blocks (one share per XCD), at least 64 slots per block
    const int64_t n_batches = (n + 63) / 64;
    int64_t grid = (int64_t)cus * 20;
    if (grid > n_batches) grid = n_batches;
    grid = (grid + kQueues - 1) / kQueues * kQueues;
    hipLaunchKernelGGL(kfn, dim3((unsigned)grid), dim3(64), 0, st, a, taylor);
    return hipGetLastError();
}

}  // namespace anf

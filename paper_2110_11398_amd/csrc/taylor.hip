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
// Work is cut by particle, not by cell: a wave takes 64 consecutive slots of
// the cell-sorted layout, so every wave carries the same work whatever the
// occupancy of the cells (a halo core spans many waves, a sparse region packs
// several cells into one).  The coefficients of the contiguous range of cells
// the 64 slots cover are staged in LDS (kTyCells cells at a time) and each lane
// reads its own cell's block.  Waves on one XCD take one contiguous run of
// slot batches, so neighbouring batches that share a cell's coefficients share
// that XCD's L2.
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
constexpr int kTyStageBytes = 8192;   // LDS per wave for staged coefficients (20 waves per CU)

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

template <int P>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(P >= 9 ? 2 : 4, 8))) void k_taylor(TyArgs a) {
    constexpr int NC = (P + 1) * (P + 2) * (P + 3) / 6;
    constexpr int kCells = kTyStageBytes / (NC * 8) > 0 ? kTyStageBytes / (NC * 8) : 1;
    __shared__ double tc[kCells * NC];
    const int lane = threadIdx.x;
    // XCD-aware contiguous chunks: block i runs on XCD i % 8; the blocks of one XCD take adjacent chunks
    const int64_t n_batches = (a.n + 63) >> 6;
    const unsigned G = gridDim.x;
    const unsigned per_xcd = G / kQueues;
    const unsigned vb = (blockIdx.x % kQueues) * per_xcd + blockIdx.x / kQueues;
    const int64_t chunk = (n_batches + G - 1) / G;
    const int64_t b_begin = (int64_t)vb * chunk;
    const int64_t b_end = b_begin + chunk < n_batches ? b_begin + chunk : n_batches;
    for (int64_t bt = b_begin; bt < b_end; bt++) {
        const int64_t slot = bt * 64 + lane;
        const bool live = slot < a.n;
        const int key = live ? a.keys[slot] : -1;
        const int c_lo = __builtin_amdgcn_readfirstlane(key);       // lane 0 is always live
        const int64_t last = (bt * 64 + 64 < a.n ? bt * 64 + 64 : a.n) - 1;
        const int c_hi = a.keys[last];
        double u = 0.0, v = 0.0, w = 0.0, s = 0.0;
        if (live) {
            const float4 sp = a.spos[slot];
            u = sp.x;
            v = sp.y;
            w = sp.z;
            const int bi = a.n_boxes > 1 ? box_of_cell(a.boxes, a.n_boxes, key) : 0;
            s = a.boxes[bi].s;
        }
        double gx = 0.0, gy = 0.0, gz = 0.0;
        for (int c0 = c_lo; c0 <= c_hi; c0 += kCells) {
            const int nc = c_hi - c0 + 1 < kCells ? c_hi - c0 + 1 : kCells;
            wave_sync();
            const double *src = a.taylor + (int64_t)c0 * NC;
            for (int i = lane; i < nc * NC; i += 64) tc[i] = src[i];
            wave_sync();
            if (live && key >= c0 && key < c0 + nc) {
                const double *T = tc + (key - c0) * NC;
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
                        // keep each column's LDS reads next to their use (no hoisting of all of them)
                        __builtin_amdgcn_sched_barrier(0);
                    }
                }
            }
        }
        if (live) {
            float *o = a.acc + 3 * (int64_t)a.perm[slot];
            o[0] = (float)((double)o[0] - s * gx);
            o[1] = (float)((double)o[1] - s * gy);
            o[2] = (float)((double)o[2] - s * gz);
        }
    }
}

typedef void (*TyKernel)(TyArgs);

template <int P>
TyKernel pick_taylor(int p) {
    if constexpr (P > kTyMaxOrder) {
        return nullptr;
    } else {
        return p == P ? k_taylor<P> : pick_taylor<P + 1>(p);
    }
}

}  // namespace

int taylor_max_order() { return kTyMaxOrder; }

hipError_t launch_taylor(const float4 *spos, const int32_t *keys, const int32_t *perm, const BoxDev *boxes,
                         int n_boxes, int64_t n, int p, const double *taylor, float *acc, int device,
                         hipStream_t st) {
    if (n <= 0) return hipSuccess;
    TyKernel kfn = pick_taylor<0>(p);
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
    // a multiple of 8 blocks (one share per XCD), at most one 64-slot batch per block
    const int64_t n_batches = (n + 63) / 64;
    int64_t grid = (int64_t)cus * 16;
    if (grid > n_batches) grid = n_batches;
    grid = (grid + kQueues - 1) / kQueues * kQueues;
    hipLaunchKernelGGL(kfn, dim3((unsigned)grid), dim3(64), 0, st, a);
    return hipGetLastError();
}

}  // namespace anf

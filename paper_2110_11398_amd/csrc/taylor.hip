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
// One wave per cell: the cell's coefficients are staged in LDS and read as
// broadcasts; each lane evaluates one particle.  For every column (b, k) the
// polynomial P_bk(u) = sum_a T^(a,b,k) u^a and its derivative come from one
// Horner pass, then
//     d/du Phi = sum P'_bk v^b w^k,  d/dv Phi = sum P_bk b v^(b-1) w^k,
//     d/dw Phi = sum P_bk v^b k w^(k-1),
// all in FP64 with the order p a compile-time constant, so every power stays
// in registers.
#include "nf_internal.h"

namespace anf {

namespace {

constexpr int kTyWaves = 2;
constexpr int kTyMaxOrder = 10;
constexpr int kTyMaxComp = (kTyMaxOrder + 1) * (kTyMaxOrder + 2) * (kTyMaxOrder + 3) / 6;

// Position of component (a, b, k) in the degree / a-descending / b-descending order.
__host__ __device__ constexpr int comp_index(int a, int b, int k) {
    const int n = a + b + k;
    return n * (n + 1) * (n + 2) / 6 + (n - a) * (n - a + 1) / 2 + (n - a - b);
}

struct TyArgs {
    const float4 *spos;
    const int32_t *cs;
    const int32_t *perm;
    const BoxDev *boxes;
    int n_boxes;
    int64_t n_cells;
    const double *taylor;
    float *acc;
};

template <int P>
__global__ __launch_bounds__(64 * kTyWaves) void k_taylor(TyArgs a) {
    constexpr int NC = (P + 1) * (P + 2) * (P + 3) / 6;
    __shared__ double tc[kTyWaves][NC > 0 ? NC : 1];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    double *T = tc[wave];
    const int64_t wave_id = (int64_t)blockIdx.x * kTyWaves + wave;
    const int64_t n_waves = (int64_t)gridDim.x * kTyWaves;
    for (int64_t c = wave_id; c < a.n_cells; c += n_waves) {
        const int cs0 = a.cs[c], n = a.cs[c + 1] - cs0;
        if (n == 0) continue;
        for (int q = lane; q < NC; q += 64) T[q] = a.taylor[c * NC + q];
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        const int bi = a.n_boxes > 1 ? box_of_cell(a.boxes, a.n_boxes, (int32_t)c) : 0;
        const double s = a.boxes[bi].s;
        for (int j0 = 0; j0 < n; j0 += 64) {
            if (j0 + lane < n) {
                const int slot = cs0 + j0 + lane;
                const float4 sp = a.spos[slot];
                const double u = sp.x, v = sp.y, w = sp.z;
                double pv[P + 1], pw[P + 1];
                pv[0] = pw[0] = 1.0;
#pragma unroll
                for (int q = 1; q <= P; q++) {
                    pv[q] = pv[q - 1] * v;
                    pw[q] = pw[q - 1] * w;
                }
                double gx = 0.0, gy = 0.0, gz = 0.0;
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
                    }
                }
                float *o = a.acc + 3 * (int64_t)a.perm[slot];
                o[0] = (float)((double)o[0] - s * gx);
                o[1] = (float)((double)o[1] - s * gy);
                o[2] = (float)((double)o[2] - s * gz);
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
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

hipError_t launch_taylor(const float4 *spos, const int32_t *cs, const int32_t *perm, const BoxDev *boxes,
                         int n_boxes, int64_t n_cells, int p, const double *taylor, float *acc, int device,
                         hipStream_t st) {
    if (n_cells <= 0) return hipSuccess;
    TyKernel kfn = pick_taylor<0>(p);
    if (!kfn) return hipErrorInvalidValue;
    TyArgs a;
    a.spos = spos;
    a.cs = cs;
    a.perm = perm;
    a.boxes = boxes;
    a.n_boxes = n_boxes;
    a.n_cells = n_cells;
    a.taylor = taylor;
    a.acc = acc;
    int cus = 1;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || cus < 1) cus = 1;
    const int64_t want = (n_cells + kTyWaves - 1) / kTyWaves;
    const int64_t cap = (int64_t)cus * 32;
    const unsigned grid = (unsigned)(want < cap ? want : cap);
    hipLaunchKernelGGL(kfn, dim3(grid), dim3(64 * kTyWaves), 0, st, a);
    return hipGetLastError();
}

}  // namespace anf

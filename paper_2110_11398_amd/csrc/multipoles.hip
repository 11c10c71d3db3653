// Cell multipole moments from the cell-sorted layout.
//
// Sec. 3.1: the far field is represented by Taylor series whose coefficients
// come from convolving the multipole moments of the mass in every cell with
// the derivatives tensor; AbacusSummit uses order p = 8.  In the paper this
// step runs on the CPU ("Compute Multipoles", Table "tbl:timing").  Here it
// reads the cell-relative coordinates that build_cells already produced:
//
//     M_c^(a,b,k) = m * sum_{j in c} u_j^a v_j^b w_j^k,   a + b + k <= p,
//
// (u, v, w) = position relative to the cell centre in cell widths.  One wave
// per cell: every lane owns up to kMaxPerLane components; particles are taken
// 64 at a time, each lane writes the powers of one particle to LDS, and every
// lane then adds the particles of the batch to its components in slot order
// (FP64 throughout, so the result does not depend on scheduling).
#include "nf_internal.h"

namespace anf {

namespace {

constexpr int kMpWaves = 2;   // 2 x 64 lanes x 33 doubles of power tables = 33.8 KB of LDS
constexpr int kMaxOrder = 10;
constexpr int kMaxComp = (kMaxOrder + 1) * (kMaxOrder + 2) * (kMaxOrder + 3) / 6;  // 286
constexpr int kMaxPerLane = (kMaxComp + 63) / 64;                                    // 5

struct MpArgs {
    const float4 *spos;
    const int32_t *cs;
    const BoxDev *boxes;
    const double *mass;  // per box (device copy)
    int n_boxes;
    int64_t n_cells;
    int p;
    int ncomp;
    double *out;
};

constexpr int kMpChunk = 24;
struct MassChunk {
    double m[kMpChunk];
    int first, count;
};

__global__ void k_set_mass(MassChunk c, double *dst) {
    int i = threadIdx.x;
    if (i < c.count) dst[c.first + i] = c.m[i];
}

__global__ __launch_bounds__(64 * kMpWaves) void k_multipoles(MpArgs a) {
    __shared__ double powt[kMpWaves][64][3 * (kMaxOrder + 1)];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int P = a.p, P1 = P + 1;
    double(*pt)[3 * (kMaxOrder + 1)] = powt[wave];

    // exponents of this lane's components: degree n, then a = n..0, then b = n-a..0
    int ea[kMaxPerLane], eb[kMaxPerLane], ek[kMaxPerLane];
    int nmine = 0;
    {
        int idx = 0;
        for (int n = 0; n <= P; n++)
            for (int x = n; x >= 0; x--)
                for (int y = n - x; y >= 0; y--, idx++)
                    if (idx % 64 == lane && nmine < kMaxPerLane) {
                        ea[nmine] = x;
                        eb[nmine] = y;
                        ek[nmine] = n - x - y;
                        nmine++;
                    }
    }

    const int64_t wave_id = (int64_t)blockIdx.x * kMpWaves + wave;
    const int64_t n_waves = (int64_t)gridDim.x * kMpWaves;
    for (int64_t c = wave_id; c < a.n_cells; c += n_waves) {
        const int cs0 = a.cs[c], n = a.cs[c + 1] - cs0;
        double acc[kMaxPerLane];
#pragma unroll
        for (int q = 0; q < kMaxPerLane; q++) acc[q] = 0.0;
        for (int j0 = 0; j0 < n; j0 += 64) {
            const int nb = min(64, n - j0);
            if (lane < nb) {
                const float4 s = a.spos[cs0 + j0 + lane];
                const double t[3] = {(double)s.x, (double)s.y, (double)s.z};
                for (int d = 0; d < 3; d++) {
                    double v = 1.0;
                    pt[lane][d * P1] = 1.0;
                    for (int q = 1; q <= P; q++) {
                        v = v * t[d];
                        pt[lane][d * P1 + q] = v;
                    }
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
            for (int j = 0; j < nb; j++) {
#pragma unroll
                for (int q = 0; q < kMaxPerLane; q++)
                    if (q < nmine) acc[q] += (pt[j][ea[q]] * pt[j][P1 + eb[q]]) * pt[j][2 * P1 + ek[q]];
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        }
        const int b = a.n_boxes > 1 ? box_of_cell(a.boxes, a.n_boxes, (int32_t)c) : 0;
        const double m = a.mass[b];
        double *o = a.out + c * a.ncomp;
#pragma unroll
        for (int q = 0; q < kMaxPerLane; q++)
            if (q < nmine) o[lane + 64 * q] = m * acc[q];
    }
}

}  // namespace

int multipole_components(int p) { return (p + 1) * (p + 2) * (p + 3) / 6; }

int multipole_max_order() { return kMaxOrder; }

hipError_t launch_multipoles(const float4 *spos, const int32_t *cs, const BoxDev *boxes, int n_boxes,
                             int64_t n_cells, int p, const double *mass_host, double *mass_dev, double *out,
                             int device, hipStream_t st) {
    for (int first = 0; first < n_boxes; first += kMpChunk) {
        MassChunk ch;
        ch.first = first;
        ch.count = n_boxes - first < kMpChunk ? n_boxes - first : kMpChunk;
        for (int k = 0; k < kMpChunk; k++) ch.m[k] = k < ch.count ? mass_host[first + k] : 0.0;
        hipLaunchKernelGGL(k_set_mass, dim3(1), dim3(kMpChunk), 0, st, ch, mass_dev);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (n_cells <= 0) return hipSuccess;
    MpArgs a;
    a.spos = spos;
    a.cs = cs;
    a.boxes = boxes;
    a.mass = mass_dev;
    a.n_boxes = n_boxes;
    a.n_cells = n_cells;
    a.p = p;
    a.ncomp = multipole_components(p);
    a.out = out;
    int cus = 1;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || cus < 1) cus = 1;
    const int64_t want = (n_cells + kMpWaves - 1) / kMpWaves;
    const int64_t cap = (int64_t)cus * 16;
    const unsigned grid = (unsigned)(want < cap ? want : cap);
    hipLaunchKernelGGL(k_multipoles, dim3(grid), dim3(64 * kMpWaves), 0, st, a);
    return hipGetLastError();
}

}  // namespace anf

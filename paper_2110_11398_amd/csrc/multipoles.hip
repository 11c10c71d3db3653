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
// (u, v, w) = position relative to the cell centre in cell widths.  Work is cut
// into units of at most kMpTile particles of one cell (a cell with more
// particles -- a halo core -- becomes several units, so no single wave serialises
// it).  One wave per unit: every lane owns up to kMaxPerLane components;
// particles are taken 64 at a time, each lane writes the powers of one particle
// to LDS, and every lane then adds the particles of the batch to its components
// in slot order.  A single-unit cell writes its moments directly; the units of
// a heavy cell write partial moments that k_mp_combine adds in unit order.
// FP64 throughout and fixed orders, so the result does not depend on scheduling.
#include "nf_internal.h"

namespace anf {

namespace {

constexpr int kMpWaves = 2;   // 2 x 64 lanes x 33 doubles of power tables = 33.8 KB of LDS
constexpr int kMaxOrder = 10;
constexpr int kMaxComp = (kMaxOrder + 1) * (kMaxOrder + 2) * (kMaxOrder + 3) / 6;  // 286
constexpr int kMaxPerLane = (kMaxComp + 63) / 64;                                    // 5

constexpr int kMpTile = 2048;  // particles per work unit

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
    const int64_t *unit_base;   // [n_cells] first unit of each cell (exclusive scan of units per cell)
    const int64_t *heavy_base;  // [n_cells] first partial slot of each multi-unit cell
    const int64_t *unit_cnt;    // [n_cells] units per cell
    double *partials;           // [slots][ncomp]
};

// Units per cell (at least one, so every cell is written) and partial slots of multi-unit cells;
// multi-unit cells are also listed for the combine step.
__global__ void k_mp_units(const int32_t *__restrict__ cs, int64_t n_cells, int64_t *__restrict__ unit_cnt,
                           int64_t *__restrict__ heavy_cnt, int32_t *__restrict__ heavy_list,
                           int32_t *__restrict__ heavy_n) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n_cells) return;
    const int n = cs[c + 1] - cs[c];
    const int64_t u = n > kMpTile ? (n + kMpTile - 1) / kMpTile : 1;
    unit_cnt[c] = u;
    heavy_cnt[c] = u > 1 ? u : 0;
    if (u > 1) heavy_list[atomicAdd(heavy_n, 1)] = (int32_t)c;
}

// Cell of unit k: the last cell whose first unit is <= k.
__device__ inline int64_t cell_of_unit(const int64_t *__restrict__ base, int64_t n_cells, int64_t k) {
    int64_t lo = 0, hi = n_cells - 1;
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) >> 1;
        if (base[mid] <= k) lo = mid; else hi = mid - 1;
    }
    return lo;
}

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
    const int64_t n_units = a.unit_base[a.n_cells - 1] + a.unit_cnt[a.n_cells - 1];
    for (int64_t k = wave_id; k < n_units; k += n_waves) {
        const int64_t c = cell_of_unit(a.unit_base, a.n_cells, k);
        const int64_t t = k - a.unit_base[c];
        const int64_t units = a.unit_cnt[c];
        const int cs0 = a.cs[c], ncell = a.cs[c + 1] - cs0;
        const int first = (int)(t * kMpTile);
        const int n = min(kMpTile, ncell - first);
        double acc[kMaxPerLane];
#pragma unroll
        for (int q = 0; q < kMaxPerLane; q++) acc[q] = 0.0;
        for (int j0 = 0; j0 < n; j0 += 64) {
            const int nb = min(64, n - j0);
            if (lane < nb) {
                const float4 s = a.spos[cs0 + first + j0 + lane];
                const double tt[3] = {(double)s.x, (double)s.y, (double)s.z};
                for (int d = 0; d < 3; d++) {
                    double v = 1.0;
                    pt[lane][d * P1] = 1.0;
                    for (int q = 1; q <= P; q++) {
                        v = v * tt[d];
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
        if (units == 1) {
            const int b = a.n_boxes > 1 ? box_of_cell(a.boxes, a.n_boxes, (int32_t)c) : 0;
            const double m = a.mass[b];
            double *o = a.out + c * a.ncomp;
#pragma unroll
            for (int q = 0; q < kMaxPerLane; q++)
                if (q < nmine) o[lane + 64 * q] = m * acc[q];
        } else {
            double *o = a.partials + (a.heavy_base[c] + t) * a.ncomp;
#pragma unroll
            for (int q = 0; q < kMaxPerLane; q++)
                if (q < nmine) o[lane + 64 * q] = acc[q];
        }
    }
}

// Moments of multi-unit cells: the partial moments of their units, added in unit order.
__global__ __launch_bounds__(64) void k_mp_combine(const int32_t *__restrict__ heavy_list,
                                                   const int32_t *__restrict__ heavy_n,
                                                   const int64_t *__restrict__ heavy_base,
                                                   const int64_t *__restrict__ unit_cnt,
                                                   const double *__restrict__ partials,
                                                   const BoxDev *__restrict__ boxes, int n_boxes,
                                                   const double *__restrict__ mass, int ncomp,
                                                   double *__restrict__ out) {
    const int nh = *heavy_n;
    for (int h = blockIdx.x; h < nh; h += gridDim.x) {
        const int32_t c = heavy_list[h];
        const int64_t units = unit_cnt[c], base = heavy_base[c];
        const int b = n_boxes > 1 ? box_of_cell(boxes, n_boxes, c) : 0;
        const double m = mass[b];
        for (int q = threadIdx.x; q < ncomp; q += 64) {
            double t = 0.0;
            for (int64_t u = 0; u < units; u++) t += partials[(base + u) * ncomp + q];
            out[(int64_t)c * ncomp + q] = m * t;
        }
    }
}

}  // namespace

int multipole_components(int p) { return (p + 1) * (p + 2) * (p + 3) / 6; }

int multipole_max_order() { return kMaxOrder; }

size_t multipole_scratch_slots(int64_t n_total, int64_t n_cells) {
    // each multi-unit cell holds more than kMpTile particles and at most 2 n_c / kMpTile units
    (void)n_cells;
    return (size_t)(2 * n_total / kMpTile + 1);
}

int multipole_tile() { return kMpTile; }

hipError_t launch_multipoles(const MultipoleBuffers &mb, const float4 *spos, const int32_t *cs,
                             const BoxDev *boxes, int n_boxes, int64_t n_cells, int p, const double *mass_host,
                             double *out, int device, void *scan_temp, hipStream_t st) {
    for (int first = 0; first < n_boxes; first += kMpChunk) {
        MassChunk ch;
        ch.first = first;
        ch.count = n_boxes - first < kMpChunk ? n_boxes - first : kMpChunk;
        for (int k = 0; k < kMpChunk; k++) ch.m[k] = k < ch.count ? mass_host[first + k] : 0.0;
        hipLaunchKernelGGL(k_set_mass, dim3(1), dim3(kMpChunk), 0, st, ch, mb.mass);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (n_cells <= 0) return hipSuccess;
    hipError_t e = launch_fill_i32(mb.heavy_n, 1, 0, st);
    if (e != hipSuccess) return e;
    const unsigned gc = (unsigned)((n_cells + 255) / 256);
    hipLaunchKernelGGL(k_mp_units, dim3(gc), dim3(256), 0, st, cs, n_cells, mb.unit_cnt, mb.heavy_cnt,
                       mb.heavy_list, mb.heavy_n);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = scan_i64_add_exclusive(mb.unit_cnt, mb.unit_base, n_cells, scan_temp, st)) != hipSuccess) return e;
    if ((e = scan_i64_add_exclusive(mb.heavy_cnt, mb.heavy_base, n_cells, scan_temp, st)) != hipSuccess) return e;
    MpArgs a;
    a.spos = spos;
    a.cs = cs;
    a.boxes = boxes;
    a.mass = mb.mass;
    a.n_boxes = n_boxes;
    a.n_cells = n_cells;
    a.p = p;
    a.ncomp = multipole_components(p);
    a.out = out;
    a.unit_base = mb.unit_base;
    a.heavy_base = mb.heavy_base;
    a.unit_cnt = mb.unit_cnt;
    a.partials = mb.partials;
    int cus = 1;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || cus < 1) cus = 1;
    const unsigned grid = (unsigned)cus * 16;
    hipLaunchKernelGGL(k_multipoles, dim3(grid), dim3(64 * kMpWaves), 0, st, a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_mp_combine, dim3((unsigned)cus * 4), dim3(64), 0, st, mb.heavy_list, mb.heavy_n,
                       mb.heavy_base, mb.unit_cnt, mb.partials, boxes, n_boxes, mb.mass, a.ncomp, out);
    return hipGetLastError();
}

}  // namespace anf

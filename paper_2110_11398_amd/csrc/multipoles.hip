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
// (u, v, w) = position relative to the cell centre in cell widths.
//
// Work is cut by particle: a work unit is kMpUnit consecutive slots of the
// sorted layout, whatever cells they hold, so every unit carries the same work
// (a halo core spans several units, a sparse region packs many cells into one).
// One wave walks its unit in batches of B slots: each lane writes one
// particle's powers to LDS as x^a y^b (a + b <= p) and w^k, then every lane
// adds the particles of the batch, in slot order, to the components it owns:
// a 2 x 2 block {x^a y^b, x^a' y^b'} x {w^k, w^k+1} (a + b = a' + b'), four
// LDS reads for four FMAs.  At each cell
// boundary the wave writes the cell's moments: directly when the whole cell
// lies in the unit, else as the unit's head or tail partial, which k_mp_combine
// adds in a fixed order.  Empty cells are written as zeros by the unit holding
// the next occupied cell (or the last unit, for trailing ones).  FP64
// throughout and fixed orders, so the result does not depend on scheduling.
#include "nf_internal.h"

namespace anf {

namespace {

constexpr int kMaxOrder = 10;
constexpr int kMpUnit = 1024;   // slots per work unit
// slots per LDS power table: 32, or 16 when cells hold fewer than 16 particles on average (smaller tables,
// more waves in flight for the per-cell work; measured on the late-time workload: 13.6 -> 11.9 ms)
constexpr int kMpBatchWide = 32, kMpBatchNarrow = 16;

__device__ inline void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// Column of x^a y^b in a power-table row: rows a = 0..P, each b = 0..P-a.
__host__ __device__ constexpr int xy_index(int P1, int a, int b) { return a * P1 - a * (a - 1) / 2 + b; }

// Position of component (a, b, k) in the degree / a-descending / b-descending order.
__host__ __device__ constexpr int comp_index(int a, int b, int k) {
    const int n = a + b + k;
    return n * (n + 1) * (n + 2) / 6 + (n - a) * (n - a + 1) / 2 + (n - a - b);
}

// The components are covered by 2 x 2 blocks {x^a y^b, x^a' y^b'} x {w^k, w^k'} with a + b = a' + b' = s
// and k' = k + 1, so a lane reads at most four powers per particle for up to four products (instead of
// two reads per product).  Blocks are numbered by s, then by the pair of (a, b) entries (a descending),
// then by the pair of k; a pair may hold a single entry at the end of its range.
__host__ __device__ constexpr int mp_blocks(int P) {
    int n = 0;
    for (int s = 0; s <= P; s++) n += ((s + 2) / 2) * ((P - s + 2) / 2);
    return n;
}

// Block idx: its two (a, b) entries (the second may be absent: b2 < 0) and two k (k2 < 0 if absent).
__device__ inline void mp_block(int P, int idx, int &a1, int &b1, int &a2, int &b2, int &k1, int &k2) {
    for (int s = 0; s <= P; s++) {
        const int nx = (s + 2) / 2, nk = (P - s + 2) / 2;
        if (idx < nx * nk) {
            const int j = idx / nk, t = idx % nk;
            a1 = s - 2 * j;
            b1 = 2 * j;
            a2 = 2 * j + 1 <= s ? s - 2 * j - 1 : 0;
            b2 = 2 * j + 1 <= s ? 2 * j + 1 : -1;
            k1 = 2 * t;
            k2 = 2 * t + 1 <= P - s ? 2 * t + 1 : -1;
            return;
        }
        idx -= nx * nk;
    }
    a1 = b1 = a2 = k1 = 0;
    b2 = k2 = -1;
}

struct MpArgs {
    const float4 *spos;
    const int32_t *keys;   // cell of every slot (sorted)
    const int32_t *cs;     // first slot of every cell, [n_cells + 1]
    const BoxDev *boxes;
    const double *mass;    // per box (device copy)
    int n_boxes;
    int64_t n;             // slots
    int64_t n_cells;
    double *out;           // [n_cells][components]
    double *partials;      // [2 per unit][components]: head, tail
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

__global__ void k_zero_f64(double *p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0.0;
}

template <int P, int kMpBatch>
__global__ __launch_bounds__(64) void k_multipoles(MpArgs a) {
    constexpr int P1 = P + 1;
    constexpr int NXY = P1 * (P1 + 1) / 2;
    constexpr int ROW = NXY + P1 + 1;   // x^a y^b, then w^k, one pad double
    constexpr int NC = P1 * (P1 + 1) * (P1 + 2) / 6;
    __shared__ double tab[kMpBatch * ROW];
    const int lane = threadIdx.x;

    // this lane's blocks: table columns of the two x^a y^b and two w^k, and the four output components
    // (-1 where a block is partial, or where the lane has no block)
    constexpr int NB = mp_blocks(P);
    constexpr int BPL = (NB + 63) / 64;
    int cx1[BPL], cx2[BPL], cz1[BPL], cz2[BPL], oc[BPL][4];
#pragma unroll
    for (int r = 0; r < BPL; r++) {
        const int idx = lane + 64 * r;
        int a1 = 0, b1 = 0, a2 = 0, b2 = -1, k1 = 0, k2 = -1;
        if (idx < NB) mp_block(P, idx, a1, b1, a2, b2, k1, k2);
        const bool has = idx < NB, has_x2 = b2 >= 0, has_k2 = k2 >= 0;
        cx1[r] = xy_index(P1, a1, b1);
        cx2[r] = has_x2 ? xy_index(P1, a2, b2) : cx1[r];
        cz1[r] = NXY + k1;
        cz2[r] = has_k2 ? NXY + k2 : cz1[r];
        oc[r][0] = has ? comp_index(a1, b1, k1) : -1;
        oc[r][1] = has && has_k2 ? comp_index(a1, b1, k2) : -1;
        oc[r][2] = has && has_x2 ? comp_index(a2, b2, k1) : -1;
        oc[r][3] = has && has_x2 && has_k2 ? comp_index(a2, b2, k2) : -1;
    }
    constexpr int NBLK_LAST = NB - 64 * (BPL - 1);   // lanes holding a block in the last round

    const int64_t n_units = (a.n + kMpUnit - 1) / kMpUnit;
    const unsigned G = gridDim.x;
    const unsigned per_xcd = G / kQueues;
    const unsigned vb = (blockIdx.x % kQueues) * per_xcd + blockIdx.x / kQueues;
    const int64_t chunk = (n_units + G - 1) / G;
    const int64_t u_begin = (int64_t)vb * chunk;
    const int64_t u_end = u_begin + chunk < n_units ? u_begin + chunk : n_units;
    const double m0 = a.mass[0];

    for (int64_t u = u_begin; u < u_end; u++) {
        const int64_t s0 = u * kMpUnit;
        const int64_t s1 = s0 + kMpUnit < a.n ? s0 + kMpUnit : a.n;
        int prev_key = s0 > 0 ? a.keys[s0 - 1] : -1;          // cell of the slot before the unit
        const int after_key = s1 < a.n ? a.keys[s1] : -1;      // cell of the slot after it (-1: none)
        bool started_here = a.keys[s0] != prev_key;            // the current segment's cell began in this unit
        double acc[BPL][4];
#pragma unroll
        for (int r = 0; r < BPL; r++)
#pragma unroll
            for (int q = 0; q < 4; q++) acc[r][q] = 0.0;

        // the next batch's keys and coordinates are loaded while the current one is summed
        int key_n = lane < kMpBatch && s0 + lane < s1 ? a.keys[s0 + lane] : -2;
        float4 sp_n = lane < kMpBatch && s0 + lane < s1 ? a.spos[s0 + lane] : make_float4(0.f, 0.f, 0.f, 0.f);
        for (int64_t b0 = s0; b0 < s1; b0 += kMpBatch) {
            const int nb = (int)(s1 - b0 < kMpBatch ? s1 - b0 : kMpBatch);
            const bool live = lane < nb;
            const int key = key_n;
            const float4 sp = sp_n;
            const int64_t b1 = b0 + kMpBatch;
            const bool live_n = lane < kMpBatch && b1 + lane < s1;
            key_n = live_n ? a.keys[b1 + lane] : -2;
            if (live_n) sp_n = a.spos[b1 + lane];
            const int first_next = __builtin_amdgcn_readfirstlane(key_n);   // cell of slot b1 when b1 < s1
            int nxt = __shfl_down(key, 1);
            if (lane == nb - 1) nxt = (b1 < s1) ? first_next : ~key;         // the unit's end closes a segment
            const uint64_t mask = __ballot(live && key != nxt);
            if (live) {
                const double x = sp.x, y = sp.y, z = sp.z;
                double xp[P1], yp[P1];
                double *row = tab + lane * ROW;
                xp[0] = yp[0] = 1.0;
                row[NXY] = 1.0;
                double zk = 1.0;
#pragma unroll
                for (int q = 1; q <= P; q++) {
                    xp[q] = xp[q - 1] * x;
                    yp[q] = yp[q - 1] * y;
                    zk = zk * z;
                    row[NXY + q] = zk;
                }
#pragma unroll
                for (int ea = 0; ea <= P; ea++)
#pragma unroll
                    for (int eb = 0; eb + ea <= P; eb++) row[xy_index(P1, ea, eb)] = xp[ea] * yp[eb];
            }
            wave_sync();
            int j = 0;
            while (j < nb) {
                const uint64_t rest = mask >> j;
                const int e = rest ? j + __builtin_ctzll(rest) : nb - 1;
                for (int t = j; t <= e; t++) {
                    const double *row = tab + t * ROW;
#pragma unroll
                    for (int r = 0; r < BPL; r++) {
                        if (r == BPL - 1 && lane >= NBLK_LAST) break;   // lanes without a block read nothing
                        const double x1 = row[cx1[r]], x2 = row[cx2[r]], z1 = row[cz1[r]], z2 = row[cz2[r]];
                        acc[r][0] = fma(x1, z1, acc[r][0]);
                        acc[r][1] = fma(x1, z2, acc[r][1]);
                        acc[r][2] = fma(x2, z1, acc[r][2]);
                        acc[r][3] = fma(x2, z2, acc[r][3]);
                    }
                }
                if (rest) {
                    // segment of cell c ends at slot b0 + e
                    const int c = __builtin_amdgcn_readlane(key, e);
                    const bool ends_here = (b0 + e + 1 < s1) || after_key != c;
                    if (started_here) {
                        // empty cells between the previous occupied cell and this one
                        double *z = a.out + (int64_t)(prev_key + 1) * NC;
                        const int64_t nz = (int64_t)(c - prev_key - 1) * NC;
                        for (int64_t i = lane; i < nz; i += 64) z[i] = 0.0;
                    }
                    double *o;
                    double scale = 1.0;
                    if (started_here && ends_here) {
                        o = a.out + (int64_t)c * NC;
                        scale = a.n_boxes > 1 ? a.mass[box_of_cell(a.boxes, a.n_boxes, c)] : m0;
                    } else {
                        o = a.partials + (2 * u + (started_here ? 1 : 0)) * NC;
                    }
#pragma unroll
                    for (int r = 0; r < BPL; r++)
#pragma unroll
                        for (int q = 0; q < 4; q++) {
                            if (oc[r][q] >= 0) o[oc[r][q]] = scale * acc[r][q];
                            acc[r][q] = 0.0;
                        }
                    prev_key = c;
                    started_here = true;
                }
                j = e + 1;
            }
            wave_sync();
        }
        if (s1 == a.n) {
            // trailing empty cells
            double *z = a.out + (int64_t)(prev_key + 1) * NC;
            const int64_t nz = (a.n_cells - 1 - prev_key) * NC;
            for (int64_t i = lane; i < nz; i += 64) z[i] = 0.0;
        }
    }
}

// Moments of the cells that cross unit boundaries: the tail partial of the unit where the cell begins,
// then the head partials of the units it continues into, added in a fixed order.
template <int P>
__global__ __launch_bounds__(64) void k_mp_combine(MpArgs a) {
    constexpr int P1 = P + 1;
    constexpr int NC = P1 * (P1 + 1) * (P1 + 2) / 6;
    const int64_t n_units = (a.n + kMpUnit - 1) / kMpUnit;
    for (int64_t u = 1 + blockIdx.x; u < n_units; u += gridDim.x) {
        const int c = a.keys[u * kMpUnit];
        if (a.keys[u * kMpUnit - 1] != c) continue;                          // no cell crosses here
        if (u >= 2 && a.keys[(u - 1) * kMpUnit - 1] == c) continue;          // crossed an earlier boundary
        const int64_t last = (a.cs[c + 1] - 1) / kMpUnit;                     // unit of the cell's last slot
        const double m = a.n_boxes > 1 ? a.mass[box_of_cell(a.boxes, a.n_boxes, c)] : a.mass[0];
        for (int i = threadIdx.x; i < NC; i += 64) {
            // head partials of units u..last in four interleaved running sums (loads in flight), added in
            // a fixed order
            double t0 = 0.0, t1 = 0.0, t2 = 0.0, t3 = 0.0;
            int64_t v = u;
            for (; v + 3 <= last; v += 4) {
                t0 += a.partials[(2 * v) * NC + i];
                t1 += a.partials[(2 * v + 2) * NC + i];
                t2 += a.partials[(2 * v + 4) * NC + i];
                t3 += a.partials[(2 * v + 6) * NC + i];
            }
            for (; v <= last; v++) t0 += a.partials[(2 * v) * NC + i];
            const double t = a.partials[(2 * (u - 1) + 1) * NC + i] + ((t0 + t1) + (t2 + t3));
            a.out[(int64_t)c * NC + i] = m * t;
        }
    }
}

typedef void (*MpKernel)(MpArgs);

template <int P>
void pick_mp(int p, bool narrow, MpKernel &main, MpKernel &combine) {
    if constexpr (P > kMaxOrder) {
        main = combine = nullptr;
    } else {
        if (p == P) {
            main = narrow ? k_multipoles<P, kMpBatchNarrow> : k_multipoles<P, kMpBatchWide>;
            combine = k_mp_combine<P>;
        } else {
            pick_mp<P + 1>(p, narrow, main, combine);
        }
    }
}

}  // namespace

int multipole_components(int p) { return (p + 1) * (p + 2) * (p + 3) / 6; }

int multipole_max_order() { return kMaxOrder; }

size_t multipole_partial_doubles(int64_t n_total, int p) {
    const int64_t units = (n_total + kMpUnit - 1) / kMpUnit;
    return (size_t)(2 * (units > 0 ? units : 1)) * (size_t)multipole_components(p);
}

hipError_t launch_multipoles(const float4 *spos, const int32_t *keys, const int32_t *cs, const BoxDev *boxes,
                             int n_boxes, int64_t n,
                             int64_t n_cells, int p, const double *mass_host, double *mass_dev, double *partials,
                             double *out, int device, hipStream_t st) {
    MpKernel kmain = nullptr, kcomb = nullptr;
    pick_mp<0>(p, n < 16 * n_cells, kmain, kcomb);
    if (!kmain) return hipErrorInvalidValue;
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
    int cus = 1;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || cus < 1) cus = 1;
    const int64_t ncomp = multipole_components(p);
    if (n <= 0) {
        const int64_t total = n_cells * ncomp;
        const int64_t blocks = std::min<int64_t>((total + 255) / 256, (int64_t)cus * 16);
        hipLaunchKernelGGL(k_zero_f64, dim3((unsigned)blocks), dim3(256), 0, st, out, total);
        return hipGetLastError();
    }
    MpArgs a;
    a.spos = spos;
    a.keys = keys;
    a.cs = cs;
    a.boxes = boxes;
    a.mass = mass_dev;
    a.n_boxes = n_boxes;
    a.n = n;
    a.n_cells = n_cells;
    a.out = out;
    a.partials = partials;
    // one unit per block (the dispatcher balances them), a multiple of 8 blocks
    const int64_t n_units = (n + kMpUnit - 1) / kMpUnit;
    int64_t grid = std::min<int64_t>(n_units, (int64_t)1 << 30);
    grid = (grid + kQueues - 1) / kQueues * kQueues;
    hipLaunchKernelGGL(kmain, dim3((unsigned)grid), dim3(64), 0, st, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || n_units < 2) return e;
    const int64_t cgrid = std::min<int64_t>(n_units - 1, (int64_t)cus * 8);
    hipLaunchKernelGGL(kcomb, dim3((unsigned)cgrid), dim3(64), 0, st, a);
    return hipGetLastError();
}

}  // namespace anf

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
// The sums run on the matrix cores.  Every component is a product of a "row"
// monomial and a "column" monomial, R_r C_c, taken from two sets of 16
// monomials each (a cover of the order, below), so the moments of a cell are
// entries of the 16 x 16 matrix sum_j R(j) C(j)^T -- a product with the
// particles as the inner index, four particles per v_mfma_f64_16x16x4f64.
// Orders 9 and 10 take two such tiles.  Each lane writes its particle's
// monomials to a row of LDS once per batch; a matrix step then reads one row
// and one column value per lane and tile.
//
// Work is cut by particle: a work unit is kMpUnit consecutive slots of the
// sorted layout, whatever cells they hold, so every unit carries the same work
// (a halo core spans several units, a sparse region packs many cells into one).
// At each cell boundary the wave writes the cell's moments: directly when the
// whole cell lies in the unit, else as the unit's head or tail partial, which
// k_mp_combine adds in a fixed order.  Empty cells are written as zeros by the
// unit holding the next occupied cell (or the last unit, for trailing ones).
// FP64 throughout and fixed orders, so the result does not depend on
// scheduling.
#include <utility>

#include "nf_internal.h"

namespace anf {

namespace {

constexpr int kMaxOrder = 10;
constexpr int kMpUnit = 1536;   // slots per work unit (measured: 1024, 2048 slower by 1.5 and 1%)
constexpr int kMxBatch = 32;   // slots per batch (rows of the LDS monomial table)

__device__ inline void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// Position of component (a, b, k) in the degree / a-descending / b-descending order.
__host__ __device__ constexpr int comp_index(int a, int b, int k) {
    const int n = a + b + k;
    return n * (n + 1) * (n + 2) / 6 + (n - a) * (n - a + 1) / 2 + (n - a - b);
}

__host__ __device__ constexpr int n_components(int P) { return (P + 1) * (P + 2) * (P + 3) / 6; }

// ---------------------------------------------------------------- covers
//
// A cover of order p: tiles of 16 row and 16 column monomials x^a y^b w^k
// such that every component a + b + k <= p is the product of a row and a
// column monomial of one tile (products of higher degree are computed and
// dropped).  Orders up to 7 and order 9 use the digit split
//     x^A y^B w^K = (x^a y^b) (x^4i y^4j w^K),  A = 4i + a, B = 4j + b,  a, b < 4,
// rows x^a y^b and columns x^4i y^4j w^K (4i + 4j + K <= p), cut into tiles of
// 16 columns (the same rows in each).  That split needs 22 columns at order 8
// and 34 at order 10; the covers used there (one tile of 16 x 16 for the 165
// components of order 8, two for the 286 of order 10) were found by a
// randomized search over pairs of monomial sets.  static_asserts below check
// that every cover reaches every component.
struct MxMono {
    int a, b, k;   // exponents of u, v, w; a < 0 marks an unused column (value 0)
};
constexpr int kMxMaxTiles = 2;
struct MxCover {
    int nt;
    MxMono row[kMxMaxTiles][16];
    MxMono col[kMxMaxTiles][16];
};

constexpr MxMono kMxRow8[16] = {{0, 0, 0}, {0, 0, 1}, {0, 0, 3}, {0, 0, 4}, {0, 1, 0}, {0, 1, 2}, {0, 2, 1}, {0, 3, 0},
                                {1, 0, 2}, {1, 1, 1}, {1, 2, 0}, {2, 0, 0}, {2, 0, 1}, {2, 1, 0}, {3, 0, 0}, {4, 0, 0}};
constexpr MxMono kMxCol8[16] = {{0, 0, 0}, {0, 0, 1}, {0, 0, 4}, {0, 0, 5}, {0, 2, 0}, {0, 3, 0}, {0, 4, 0}, {0, 5, 0},
                                {1, 0, 0}, {1, 0, 1}, {1, 1, 3}, {1, 2, 1}, {2, 0, 1}, {2, 2, 1}, {4, 0, 0}, {5, 0, 0}};
constexpr MxMono kMxRow10[2][16] = {
    {{0, 0, 2}, {0, 1, 1}, {0, 1, 2}, {0, 2, 0}, {0, 2, 1}, {0, 3, 0}, {1, 0, 1}, {1, 0, 2},
     {1, 1, 0}, {1, 1, 1}, {1, 2, 0}, {2, 0, 0}, {2, 0, 1}, {2, 1, 0}, {3, 0, 0}, {3, 0, 2}},
    {{0, 0, 0}, {0, 0, 1}, {0, 0, 2}, {0, 1, 0}, {0, 1, 1}, {0, 1, 2}, {0, 4, 0}, {0, 5, 3},
     {1, 0, 0}, {1, 0, 1}, {1, 1, 0}, {1, 1, 1}, {1, 2, 4}, {2, 0, 0}, {2, 2, 0}, {6, 0, 0}}};
constexpr MxMono kMxCol10[2][16] = {
    {{0, 0, 3}, {0, 0, 5}, {0, 3, 0}, {0, 4, 0}, {0, 5, 2}, {1, 1, 0}, {1, 1, 5}, {1, 3, 2},
     {2, 3, 0}, {2, 5, 0}, {3, 0, 0}, {4, 0, 3}, {4, 3, 0}, {5, 0, 0}, {5, 0, 2}, {6, 1, 0}},
    {{0, 0, 0}, {0, 0, 2}, {0, 0, 6}, {0, 0, 8}, {0, 2, 0}, {0, 2, 6}, {0, 3, 3}, {0, 6, 0},
     {0, 8, 0}, {2, 0, 0}, {2, 0, 4}, {2, 0, 6}, {2, 2, 3}, {3, 0, 3}, {3, 2, 1}, {8, 0, 0}}};

constexpr MxCover mx_cover(int P) {
    MxCover v{};
    if (P == 8) {
        v.nt = 1;
        for (int i = 0; i < 16; i++) {
            v.row[0][i] = kMxRow8[i];
            v.col[0][i] = kMxCol8[i];
        }
        return v;
    }
    if (P == 10) {
        v.nt = 2;
        for (int t = 0; t < 2; t++)
            for (int i = 0; i < 16; i++) {
                v.row[t][i] = kMxRow10[t][i];
                v.col[t][i] = kMxCol10[t][i];
            }
        return v;
    }
    // digit split
    int nc = 0;
    for (int t = 0; t < kMxMaxTiles; t++)
        for (int i = 0; i < 16; i++) v.col[t][i] = MxMono{-1, 0, 0};
    for (int i = 0; 4 * i <= P; i++)
        for (int j = 0; 4 * i + 4 * j <= P; j++)
            for (int k = 0; 4 * i + 4 * j + k <= P; k++, nc++) v.col[nc / 16][nc % 16] = MxMono{4 * i, 4 * j, k};
    v.nt = (nc + 15) / 16;
    for (int t = 0; t < v.nt; t++)
        for (int r = 0; r < 16; r++) v.row[t][r] = MxMono{r & 3, r >> 2, 0};
    return v;
}

// Component of every (tile, row, column) entry: the first entry in (tile, row, column) order whose product is
// the component stands for it; every other entry is -1.
struct MxMap {
    short comp[kMaxOrder + 1][kMxMaxTiles][16][16];
    bool complete[kMaxOrder + 1];
};

constexpr MxMap mx_map() {
    MxMap m{};
    for (int P = 0; P <= kMaxOrder; P++) {
        const MxCover cv = mx_cover(P);
        bool seen[n_components(kMaxOrder)] = {};
        for (int t = 0; t < kMxMaxTiles; t++)
            for (int r = 0; r < 16; r++)
                for (int c = 0; c < 16; c++) {
                    m.comp[P][t][r][c] = -1;
                    if (t >= cv.nt || cv.col[t][c].a < 0) continue;
                    const int A = cv.row[t][r].a + cv.col[t][c].a, B = cv.row[t][r].b + cv.col[t][c].b,
                              K = cv.row[t][r].k + cv.col[t][c].k;
                    if (A + B + K > P) continue;
                    const int ci = comp_index(A, B, K);
                    if (seen[ci]) continue;
                    seen[ci] = true;
                    m.comp[P][t][r][c] = (short)ci;
                }
        bool all = true;
        for (int i = 0; i < n_components(P); i++) all = all && seen[i];
        m.complete[P] = all;
    }
    return m;
}

constexpr MxMap kMxMapHost = mx_map();
static_assert(kMxMapHost.complete[0] && kMxMapHost.complete[1] && kMxMapHost.complete[2] &&
                  kMxMapHost.complete[3] && kMxMapHost.complete[4] && kMxMapHost.complete[5] &&
                  kMxMapHost.complete[6] && kMxMapHost.complete[7] && kMxMapHost.complete[8] &&
                  kMxMapHost.complete[9] && kMxMapHost.complete[10],
              "a multipole cover misses a component");
static_assert(mx_cover(8).nt == 1 && mx_cover(9).nt == 2 && mx_cover(10).nt == 2, "tiles per order");

__constant__ MxMap kMxMap = mx_map();

// Entry idx of a particle's LDS row (idx a compile-time constant): entries 32 t .. 32 t + 15 hold the row
// monomials of tile t, 32 t + 16 .. 32 t + 31 its column monomials.  Unused columns, and monomials of a degree
// beyond p along one axis (which reach no component), are zeros.
template <int P, int idx>
__device__ inline double mx_entry(const double (&xp)[P + 1], const double (&yp)[P + 1], const double (&zp)[P + 1]) {
    constexpr MxCover cv = mx_cover(P);
    constexpr MxMono m = (idx & 31) < 16 ? cv.row[idx >> 5][idx & 15] : cv.col[idx >> 5][idx & 15];
    if constexpr (m.a < 0 || m.a > P || m.b > P || m.k > P) {
        return 0.0;
    } else {
        return xp[m.a] * yp[m.b] * zp[m.k];
    }
}

template <int P, int... is>
__device__ inline void mx_write_row(double *row, const double (&xp)[P + 1], const double (&yp)[P + 1],
                                    const double (&zp)[P + 1], std::integer_sequence<int, is...>) {
    ((row[is] = mx_entry<P, is>(xp, yp, zp)), ...);
}

typedef double mx_acc __attribute__((ext_vector_type(4)));

// A wave-uniform double held in scalar registers.
__device__ inline double uniform_f64(double v) {
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)b);
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(b >> 32));
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
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

// STAGE: each cell's components go through LDS into component order and are written by consecutive lanes
// (whole cache lines; pays where cells are small and the per-cell output dominates), else each lane stores its
// accumulator entries directly (no LDS for it: one more wave per CU).
template <int P, int B, bool STAGE>
__global__ __launch_bounds__(64) void k_multipoles(MpArgs a) {
    constexpr int P1 = P + 1;
    constexpr int NC = n_components(P);
    constexpr int NT = mx_cover(P).nt;
    constexpr int ROW = 32 * NT + 2;   // per tile 16 row and 16 column monomials; pad (16-byte rows)
    // B rows written every batch (finite values: lanes past the batch's end write the monomials of 0), then 3
    // zero rows, so that a step may read rows up to 3 past a segment's end without a bound
    __shared__ __align__(16) double tab[(B + 3) * ROW];
    __shared__ double out_stage[STAGE ? NC : 1];   // one cell's components in component order
    const int lane = threadIdx.x;
    const int g = lane >> 4, col = lane & 15;
    for (int i = lane; i < 3 * ROW; i += 64) tab[B * ROW + i] = 0.0;

    // The accumulator of tile t holds entry (row 4 q + g, column col) in its register q (the layout of
    // v_mfma_f64_16x16x4f64's result); component of each, or -1
    int oc[NT][4];
#pragma unroll
    for (int t = 0; t < NT; t++)
#pragma unroll
        for (int q = 0; q < 4; q++) oc[t][q] = kMxMap.comp[P][t][4 * q + g][col];

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
        mx_acc acc[NT];
#pragma unroll
        for (int t = 0; t < NT; t++) acc[t] = mx_acc{0.0, 0.0, 0.0, 0.0};

        // the next batch's keys, successor keys (-3: the unit ends after the slot) and coordinates are loaded
        // while the current one is summed
        int key_n = lane < B && s0 + lane < s1 ? a.keys[s0 + lane] : -2;
        int nxt_n = lane < B && s0 + lane + 1 < s1 ? a.keys[s0 + lane + 1] : -3;
        float4 sp_n = lane < B && s0 + lane < s1 ? a.spos[s0 + lane] : make_float4(0.f, 0.f, 0.f, 0.f);
        for (int64_t b0 = s0; b0 < s1; b0 += B) {
            const int nb = (int)(s1 - b0 < B ? s1 - b0 : B);
            const bool live = lane < nb;
            const int key = key_n, nxt = nxt_n;
            const float4 sp = sp_n;
            const int64_t b1 = b0 + B;
            const bool live_n = lane < B && b1 + lane < s1;
            key_n = live_n ? a.keys[b1 + lane] : -2;
            nxt_n = lane < B && b1 + lane + 1 < s1 ? a.keys[b1 + lane + 1] : -3;
            if (live_n) sp_n = a.spos[b1 + lane];
            const uint64_t mask = __ballot(live && key != nxt);   // slots that end a segment
            if (lane < B) {
                // this lane's particle: its row and column monomials (zeros past the batch's end)
                const double x = live ? (double)sp.x : 0.0, y = live ? (double)sp.y : 0.0,
                             z = live ? (double)sp.z : 0.0;
                double xp[P1], yp[P1], zp[P1];
                xp[0] = yp[0] = zp[0] = 1.0;
#pragma unroll
                for (int q = 1; q <= P; q++) {
                    xp[q] = xp[q - 1] * x;
                    yp[q] = yp[q - 1] * y;
                    zp[q] = zp[q - 1] * z;
                }
                mx_write_row<P>(tab + lane * ROW, xp, yp, zp, std::make_integer_sequence<int, 32 * NT>{});
            }
            wave_sync();
            int j = 0;
            while (j < nb) {
                const uint64_t rest = mask >> j;
                const int e = rest ? j + __builtin_ctzll(rest) : nb - 1;
                const double *rp = tab + (j + g) * ROW;
                for (int t0 = j; t0 <= e; t0 += 4, rp += 4 * ROW) {
                    // particle t0 + g of the step; past the segment's end its row monomials are replaced by zeros
                    double av[NT], bv[NT];
#pragma unroll
                    for (int t = 0; t < NT; t++) {
                        av[t] = rp[32 * t + col];
                        bv[t] = rp[32 * t + 16 + col];
                    }
#pragma unroll
                    for (int t = 0; t < NT; t++) {
                        av[t] = t0 + g <= e ? av[t] : 0.0;
                        acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[t], bv[t], acc[t], 0, 0, 0);
                    }
                }
                if (rest) {
                    // segment of cell c ends at slot b0 + e
                    const int c = __builtin_amdgcn_readlane(key, e);
                    const bool ends_here = (b0 + e + 1 < s1) || after_key != c;
                    if (started_here) {
                        // empty cells between the previous occupied cell and this one
                        double *zz = a.out + (int64_t)(prev_key + 1) * NC;
                        const int64_t nz = (int64_t)(c - prev_key - 1) * NC;
                        for (int64_t i = lane; i < nz; i += 64) zz[i] = 0.0;
                    }
                    double *o;
                    double scale = 1.0;
                    if (started_here && ends_here) {
                        o = a.out + (int64_t)c * NC;
                        scale = a.n_boxes > 1 ? a.mass[box_of_cell(a.boxes, a.n_boxes, c)] : m0;
                    } else {
                        o = a.partials + (2 * u + (started_here ? 1 : 0)) * NC;
                    }
                    scale = uniform_f64(scale);   // waited for here, not at every store below
                    if constexpr (STAGE) {
#pragma unroll
                        for (int t = 0; t < NT; t++) {
#pragma unroll
                            for (int q = 0; q < 4; q++)
                                if (oc[t][q] >= 0) out_stage[oc[t][q]] = scale * acc[t][q];
                            acc[t] = mx_acc{0.0, 0.0, 0.0, 0.0};
                        }
                        wave_sync();
                        for (int i = lane; i < NC; i += 64) o[i] = out_stage[i];
                        wave_sync();
                    } else {
                        double v[NT][4];
#pragma unroll
                        for (int t = 0; t < NT; t++) {
#pragma unroll
                            for (int q = 0; q < 4; q++) v[t][q] = scale * acc[t][q];
                            acc[t] = mx_acc{0.0, 0.0, 0.0, 0.0};
                        }
#pragma unroll
                        for (int t = 0; t < NT; t++)
#pragma unroll
                            for (int q = 0; q < 4; q++)
                                if (oc[t][q] >= 0) o[oc[t][q]] = v[t][q];
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
            double *zz = a.out + (int64_t)(prev_key + 1) * NC;
            const int64_t nz = (a.n_cells - 1 - prev_key) * NC;
            for (int64_t i = lane; i < nz; i += 64) zz[i] = 0.0;
        }
    }
}

// Moments of the cells that cross unit boundaries: the tail partial of the unit where the cell begins,
// then the head partials of the units it continues into, added in a fixed order.  One workgroup per boundary:
// wave w sums the head partials of units u + w, u + w + 4, ... in four interleaved running sums (a halo core
// spans tens of units, so sixteen partials' loads are in flight at a time), and the first wave adds the four
// waves' sums in a fixed order.
template <int P>
__global__ __launch_bounds__(256) void k_mp_combine(MpArgs a) {
    constexpr int NC = n_components(P);
    __shared__ double part[4][NC];
    const int64_t n_units = (a.n + kMpUnit - 1) / kMpUnit;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int64_t u = 1 + blockIdx.x; u < n_units; u += gridDim.x) {
        // the same u for the whole workgroup: the tests below are uniform
        const int c = a.keys[u * kMpUnit];
        if (a.keys[u * kMpUnit - 1] != c) continue;                          // no cell crosses here
        if (u >= 2 && a.keys[(u - 1) * kMpUnit - 1] == c) continue;          // crossed an earlier boundary
        const int64_t last = (a.cs[c + 1] - 1) / kMpUnit;                     // unit of the cell's last slot
        for (int i = lane; i < NC; i += 64) {
            double t0 = 0.0, t1 = 0.0, t2 = 0.0, t3 = 0.0;
            int64_t v = u + w;
            for (; v + 12 <= last; v += 16) {
                t0 += a.partials[(2 * v) * NC + i];
                t1 += a.partials[(2 * v + 8) * NC + i];
                t2 += a.partials[(2 * v + 16) * NC + i];
                t3 += a.partials[(2 * v + 24) * NC + i];
            }
            for (; v <= last; v += 4) t0 += a.partials[(2 * v) * NC + i];
            part[w][i] = (t0 + t1) + (t2 + t3);
        }
        __syncthreads();
        if (w == 0) {
            const double m = a.n_boxes > 1 ? a.mass[box_of_cell(a.boxes, a.n_boxes, c)] : a.mass[0];
            for (int i = lane; i < NC; i += 64) {
                const double heads = (part[0][i] + part[1][i]) + (part[2][i] + part[3][i]);
                a.out[(int64_t)c * NC + i] = m * (a.partials[(2 * (u - 1) + 1) * NC + i] + heads);
            }
        }
        __syncthreads();
    }
}

typedef void (*MpKernel)(MpArgs);

template <int P>
void pick_mp(int p, bool stage, MpKernel &main, MpKernel &combine) {
    if constexpr (P > kMaxOrder) {
        main = combine = nullptr;
    } else {
        if (p == P) {
            main = stage ? k_multipoles<P, kMxBatch, true> : k_multipoles<P, kMxBatch, false>;
            combine = k_mp_combine<P>;
        } else {
            pick_mp<P + 1>(p, stage, main, combine);
        }
    }
}

}  // namespace

int multipole_components(int p) { return n_components(p); }

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
    // cells of fewer than 16 particles on average: the per-cell output dominates, stage it (measured on the
    // late-time workload, 8 per cell: 9.33 -> 8.47 ms; on the clustered one, 64 per cell, staging costs 5%)
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
    const int64_t cgrid = std::min<int64_t>(n_units - 1, (int64_t)1 << 20);   // a boundary per workgroup
    hipLaunchKernelGGL(kcomb, dim3((unsigned)cgrid), dim3(256), 0, st, a);
    return hipGetLastError();
}

}  // namespace anf

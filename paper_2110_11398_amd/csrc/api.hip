// C ABI of libabacus_nf: argument checks, buffer management, and the launch
// sequence of each entry point.  Every argument check runs before the first
// HIP call, so invalid calls fail synchronously without touching the device.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "nf_internal.h"

using namespace anf;

struct abacus_nf_cells_s {
    int device = -1;
    int64_t n_total = 0, n_cells = 0;
    int32_t n_boxes = 0, R = 2;
    bool built = false;
    std::vector<abacus_nf_box> boxes;
    std::vector<int32_t> cell_base;
    abacus_nf_tuning tune{};

    // capacities (elements)
    int64_t cap_n = -1, cap_cells = -1, cap_boxes = -1;
    int32_t *keys_a = nullptr, *vals_a = nullptr, *keys_b = nullptr, *vals_b = nullptr;
    int32_t *keys = nullptr, *perm = nullptr;  // sorted results (point into the buffers above)
    float4 *spos = nullptr;
    int32_t *cell_start = nullptr;
    int32_t *endpos = nullptr;
    void *radix_temp = nullptr;
    void *scan_temp = nullptr;
    BoxDev *d_boxes = nullptr;
    double *d_mass = nullptr;  // per-box mass for the multipoles
    // partial moments of the multipole work units (allocated by the first multipoles call that needs more)
    size_t mp_cap = 0;
    double *mp_partials = nullptr;

    // leapfrog: per-box step sizes (kick, drift), timestep partials and per-box minima
    int scap_boxes = -1;
    double *d_dt = nullptr;                 // [2][n_boxes]
    unsigned long long *ts_min = nullptr;   // timestep_min_words(n_boxes): per-box slots, then final minima
    size_t ts_cap = 0;
    double *ts_partials = nullptr;
    // merge scratch (n_total x 12 bytes)
    size_t merge_cap = 0;
    void *merge_tmp = nullptr;

    // force work buffers
    int64_t wcap_cells = -1, wcap_items = -1, wcap_partials = -1, wcap_boxes = -1;
    ForceBox *d_fbox = nullptr;
    WorkState *ws = nullptr;
    Item *items = nullptr;
    int32_t *cell_nsrc = nullptr, *cell_parts = nullptr;
    int64_t *cell_pdem = nullptr, *cell_pbase = nullptr;
    double *partials = nullptr;
    void *wscan_temp = nullptr;
    // largest |a|^2 per cell (bits of a non-negative double) written by the last forces call; valid until
    // the next build
    unsigned long long *cell_amax = nullptr;
    bool amax_valid = false;

    // persistent-kernel grid of the last (kind, mode, tuning): queried once, outside any capture
    int grid = 0;
    int grid_key[8] = {-1, -1, -1, -1, -1, -1, -1, -1};

    // optional stage timing: event pairs for build, work list, kernel, finalize
    bool timing = false;
    hipEvent_t ev[8] = {nullptr};
    bool ev_used[4] = {false, false, false, false};
};

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_err_mutex;
int *g_err[kMaxDevices] = {nullptr};

template <typename T>
void dfree(T *&p) {
    if (p) hipFree((void *)p);
    p = nullptr;
}

template <typename T>
bool dalloc(T *&p, size_t count) {
    dfree(p);
    if (count == 0) count = 1;
    void *q = nullptr;
    if (hipMalloc(&q, count * sizeof(T)) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    p = (T *)q;
    return true;
}

bool dalloc_bytes(void *&p, size_t bytes) {
    if (p) hipFree(p);
    p = nullptr;
    if (hipMalloc(&p, bytes ? bytes : 1) != hipSuccess) {
        (void)hipGetLastError();
        p = nullptr;
        return false;
    }
    return true;
}

void free_sort_buffers(abacus_nf_cells_s *h) {
    dfree(h->keys_a); dfree(h->vals_a); dfree(h->keys_b); dfree(h->vals_b);
    dfree(h->spos); dfree(h->cell_start); dfree(h->endpos); dfree(h->d_boxes); dfree(h->d_mass);
    if (h->radix_temp) hipFree(h->radix_temp);
    if (h->scan_temp) hipFree(h->scan_temp);
    h->radix_temp = h->scan_temp = nullptr;
    h->keys = h->perm = nullptr;
    h->cap_n = h->cap_cells = h->cap_boxes = -1;
}

void destroy_events(abacus_nf_cells_s *h) {
    for (int i = 0; i < 8; i++)
        if (h->ev[i]) hipEventDestroy(h->ev[i]);
    for (int i = 0; i < 8; i++) h->ev[i] = nullptr;
    for (int i = 0; i < 4; i++) h->ev_used[i] = false;
}

void mark(abacus_nf_cells_s *h, int stage, bool end, hipStream_t st) {
    if (!h->timing || !h->ev[2 * stage + (end ? 1 : 0)]) return;
    hipEventRecord(h->ev[2 * stage + (end ? 1 : 0)], st);
    if (end) h->ev_used[stage] = true;
}

void free_mp_buffers(abacus_nf_cells_s *h) {
    dfree(h->mp_partials);
    h->mp_cap = 0;
}

void free_step_buffers(abacus_nf_cells_s *h) {
    dfree(h->d_dt);
    dfree(h->ts_min);
    dfree(h->ts_partials);
    h->scap_boxes = -1;
    h->ts_cap = 0;
    if (h->merge_tmp) hipFree(h->merge_tmp);
    h->merge_tmp = nullptr;
    h->merge_cap = 0;
}

void free_work_buffers(abacus_nf_cells_s *h) {
    dfree(h->d_fbox); dfree(h->ws); dfree(h->items); dfree(h->cell_nsrc); dfree(h->cell_parts);
    dfree(h->cell_pdem); dfree(h->cell_pbase); dfree(h->partials); dfree(h->cell_amax);
    h->amax_valid = false;
    if (h->wscan_temp) hipFree(h->wscan_temp);
    h->wscan_temp = nullptr;
    h->wcap_cells = h->wcap_items = h->wcap_partials = h->wcap_boxes = -1;
}

int key_bits(int64_t n_cells) {
    int b = 0;
    while (((int64_t)1 << b) < n_cells) b++;
    return b;
}

abacus_nf_tuning default_tuning() {
    abacus_nf_tuning t;
    memset(&t, 0, sizeof(t));
    t.sinks_per_lane = 2;
    t.chunk = 256;
    t.unroll = 2;
    t.max_lanes = 64;
    t.part_sources = 1 << 16;
    t.waves_per_cu = 0;
    t.item_capacity = 0;
    return t;
}

// Resolve zero fields to defaults; return false if a field is out of range.
bool resolve_tuning(const abacus_nf_tuning *in, abacus_nf_tuning *out) {
    abacus_nf_tuning d = default_tuning();
    abacus_nf_tuning t = in ? *in : d;
    if (!t.sinks_per_lane) t.sinks_per_lane = d.sinks_per_lane;
    if (!t.chunk) t.chunk = d.chunk;
    if (!t.unroll) t.unroll = d.unroll;
    if (!t.max_lanes) t.max_lanes = d.max_lanes;
    if (!t.part_sources) t.part_sources = d.part_sources;
    if (t.sinks_per_lane != 1 && t.sinks_per_lane != 2 && t.sinks_per_lane != 4) return false;
    if (t.unroll != 1 && t.unroll != 2 && t.unroll != 4) return false;
    if (t.chunk % 64 != 0 || t.chunk < 64 * t.unroll || t.chunk > 512) return false;
    if (t.max_lanes < 1 || t.max_lanes > 64) return false;
    if (t.part_sources < 1024) return false;
    if (t.waves_per_cu < 0 || t.waves_per_cu > 64) return false;
    if (t.occupancy != 0 && t.occupancy != 6 && t.occupancy != 8) return false;
    if (t.reserved != 0) return false;
    if (t.item_capacity < 0 || t.item_capacity >= INT32_MAX) return false;
    *out = t;
    return true;
}

int hip_fail(hipError_t e) {
    (void)e;
    (void)hipGetLastError();
    return ABACUS_NF_EDEVICE;
}

}  // namespace

namespace anf {

int *device_error_word(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_err_mutex);
    if (!g_err[device]) {
        void *p = nullptr;
        if (hipMalloc(&p, sizeof(int)) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        if (hipMemset(p, 0, sizeof(int)) != hipSuccess) {
            (void)hipGetLastError();
            hipFree(p);
            return nullptr;
        }
        g_err[device] = (int *)p;
    }
    return g_err[device];
}

}  // namespace anf

extern "C" {

int abacus_nf_version(void) { return 1 * 10000 + 0 * 100 + 0; }

const char *abacus_nf_strerror(int code) {
    switch (code) {
        case ABACUS_NF_OK: return "ok";
        case ABACUS_NF_EINVAL: return "invalid argument";
        case ABACUS_NF_ENOMEM: return "out of memory";
        case ABACUS_NF_EDEVICE: return "HIP runtime error";
        case ABACUS_NF_ECAPACITY: return "device work list outgrew its capacity";
        case ABACUS_NF_ENONFINITE: return "non-finite particle position";
        case ABACUS_NF_ESTATE: return "handle used in the wrong state";
        case ABACUS_NF_ELIMIT: return "batch exceeds the fixed scratch of an entry point that allocates nothing";
        default: return "unknown error code";
    }
}

int abacus_nf_build_cells(const float *pos, int64_t n_total, const abacus_nf_box *boxes, int32_t n_boxes,
                          int32_t R, void *hip_stream, abacus_nf_cells *cells) {
    // ---- argument checks (no HIP call before this block ends)
    if (!cells || !boxes) return ABACUS_NF_EINVAL;
    if (n_total < 0 || n_total >= INT32_MAX) return ABACUS_NF_EINVAL;
    if (n_total > 0 && !pos) return ABACUS_NF_EINVAL;
    if (n_boxes < 1 || n_boxes > 65536) return ABACUS_NF_EINVAL;
    if (R < 1 || R > 3) return ABACUS_NF_EINVAL;
    std::vector<int32_t> base((size_t)n_boxes);
    int64_t off = 0, cells_total = 0;
    for (int b = 0; b < n_boxes; b++) {
        const abacus_nf_box &x = boxes[b];
        if (x.offset != off || x.n < 0 || x.reserved != 0) return ABACUS_NF_EINVAL;
        if (!(x.box > 0) || !std::isfinite(x.box)) return ABACUS_NF_EINVAL;
        if (x.K < 2 * R + 1 || x.K > 1290) return ABACUS_NF_EINVAL;
        off += x.n;
        base[b] = (int32_t)cells_total;
        cells_total += (int64_t)x.K * x.K * x.K;
        if (cells_total >= INT32_MAX) return ABACUS_NF_EINVAL;
    }
    if (off != n_total) return ABACUS_NF_EINVAL;

    // ---- buffers
    hipStream_t st = (hipStream_t)hip_stream;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return hip_fail(hipErrorUnknown);
    int *err = device_error_word(dev);
    if (!err) return ABACUS_NF_ENOMEM;
    abacus_nf_cells_s *h = *cells;
    bool fresh = false;
    if (!h) {
        h = new (std::nothrow) abacus_nf_cells_s();
        if (!h) return ABACUS_NF_ENOMEM;
        h->tune = default_tuning();
        fresh = true;
    } else if (h->device != dev) {
        return ABACUS_NF_ESTATE;
    }
    h->device = dev;
    const int64_t n = n_total;
    if (h->cap_n < n || h->cap_cells < cells_total || h->cap_boxes < n_boxes) {
        free_sort_buffers(h);
        const int64_t cn = std::max<int64_t>(n, 1), cc = std::max<int64_t>(cells_total, 1);
        bool ok = dalloc(h->keys_a, cn) && dalloc(h->vals_a, cn) && dalloc(h->keys_b, cn) &&
                  dalloc(h->vals_b, cn) && dalloc(h->spos, cn) && dalloc(h->cell_start, cc + 1) &&
                  dalloc(h->endpos, cc) && dalloc(h->d_boxes, n_boxes) && dalloc(h->d_mass, n_boxes) &&
                  dalloc_bytes(h->radix_temp, radix_temp_bytes(cn)) &&
                  dalloc_bytes(h->scan_temp, scan_temp_bytes(std::max(cc, cn)));
        if (!ok) {
            free_sort_buffers(h);
            if (fresh) delete h;
            return ABACUS_NF_ENOMEM;
        }
        h->cap_n = cn;
        h->cap_cells = cc;
        h->cap_boxes = n_boxes;
    }
    h->n_total = n;
    h->n_cells = cells_total;
    h->n_boxes = n_boxes;
    h->R = R;
    h->boxes.assign(boxes, boxes + n_boxes);
    h->cell_base = base;
    h->built = false;
    h->amax_valid = false;
    *cells = h;

    // ---- enqueue
    mark(h, 0, false, st);
    hipError_t e = launch_set_boxes(boxes, n_boxes, base.data(), h->d_boxes, st);
    if (e == hipSuccess) e = launch_bin(pos, n, h->d_boxes, n_boxes, h->keys_a, h->vals_a, err, st);
    int32_t *ks = h->keys_a, *vs = h->vals_a;
    if (e == hipSuccess)
        e = radix_sort_pairs(h->keys_a, h->vals_a, h->keys_b, h->vals_b, h->radix_temp, n, key_bits(cells_total), st,
                             &ks, &vs);
    if (e == hipSuccess) e = launch_cell_start(ks, n, cells_total, h->endpos, h->cell_start, h->scan_temp, st);
    if (e == hipSuccess) e = launch_gather(pos, vs, ks, n, h->d_boxes, n_boxes, h->spos, st);
    if (e != hipSuccess) return hip_fail(e);
    mark(h, 0, true, st);
    h->keys = ks;
    h->perm = vs;
    h->built = true;
    return ABACUS_NF_OK;
}

static int check_force_args(abacus_nf_cells h, const double *eps, abacus_nf_kind kind, const double *gm,
                            abacus_nf_sum mode, const void *acc) {
    if (!h || !eps || !gm) return ABACUS_NF_EINVAL;
    if (kind != ABACUS_NF_SPLINE && kind != ABACUS_NF_PLUMMER) return ABACUS_NF_EINVAL;
    if (mode != ABACUS_NF_SUM_FP32 && mode != ABACUS_NF_SUM_COMP32 && mode != ABACUS_NF_SUM_FP64)
        return ABACUS_NF_EINVAL;
    if (!h->built) return ABACUS_NF_ESTATE;
    if (h->n_total > 0 && !acc) return ABACUS_NF_EINVAL;
    for (int b = 0; b < h->n_boxes; b++) {
        const double w = h->boxes[b].box / h->boxes[b].K;
        if (!std::isfinite(eps[b]) || !std::isfinite(gm[b])) return ABACUS_NF_EINVAL;
        const double ec = eps[b] / w;
        if (!(ec >= 1e-5 && ec <= 1.0)) return ABACUS_NF_EINVAL;
        if (!std::isfinite(gm[b] / (w * w))) return ABACUS_NF_EINVAL;
    }
    return ABACUS_NF_OK;
}

static int ensure_work_buffers(abacus_nf_cells_s *h) {
    const int64_t n = std::max<int64_t>(h->n_total, 1);
    const int64_t nc = std::max<int64_t>(h->n_cells, 1);
    // unsplit items: one tile per non-empty cell, one per 64 sink groups, and at most one more per 11
    // groups of a cell's rest (its binary cut); split source lists take the rest of the capacity
    const int64_t want_items = h->tune.item_capacity > 0
                                   ? h->tune.item_capacity
                                   : std::min<int64_t>(INT32_MAX - 1, std::min(n, nc) + n / 16 + n / 11 + (1 << 16));
    const int64_t want_partials = 2 * n + (1 << 16);
    if (h->wcap_cells >= nc && h->wcap_items == want_items && h->wcap_partials >= want_partials &&
        h->wcap_boxes >= h->n_boxes)
        return ABACUS_NF_OK;
    free_work_buffers(h);
    bool ok = dalloc(h->d_fbox, h->n_boxes) && dalloc(h->ws, 1) && dalloc(h->items, want_items) &&
              dalloc(h->cell_nsrc, nc) && dalloc(h->cell_parts, nc) && dalloc(h->cell_pdem, nc) &&
              dalloc(h->cell_pbase, nc) && dalloc(h->partials, 4 * want_partials) && dalloc(h->cell_amax, nc) &&
              dalloc_bytes(h->wscan_temp, scan_temp_bytes(nc));
    if (!ok) {
        free_work_buffers(h);
        return ABACUS_NF_ENOMEM;
    }
    h->wcap_cells = nc;
    h->wcap_items = want_items;
    h->wcap_partials = want_partials;
    h->wcap_boxes = h->n_boxes;
    return ABACUS_NF_OK;
}

static ForcesArgs make_args(abacus_nf_cells_s *h, abacus_nf_kind kind, abacus_nf_sum mode, float *acc, int *err) {
    ForcesArgs a;
    memset(&a, 0, sizeof(a));
    a.spos = h->spos;
    a.cell_start = h->cell_start;
    a.perm = h->perm;
    a.keys = h->keys;
    a.boxes = h->d_boxes;
    a.fbox = h->d_fbox;
    a.n_boxes = h->n_boxes;
    a.n_total = h->n_total;
    a.n_cells = h->n_cells;
    a.R = h->R;
    a.items = h->items;
    a.item_capacity = h->wcap_items;
    a.ws = h->ws;
    a.cell_nsrc = h->cell_nsrc;
    a.cell_parts = h->cell_parts;
    a.cell_pdem = h->cell_pdem;
    a.cell_pbase = h->cell_pbase;
    a.partials = h->partials;
    a.partial_capacity = h->wcap_partials;
    a.amax = h->cell_amax;
    a.acc = acc;
    a.rho = nullptr;
    a.err = err;
    a.kind = kind;
    a.mode = mode;
    a.tune = h->tune;
    a.scan_temp = h->wscan_temp;
    return a;
}

static int forces_impl(abacus_nf_cells h, const double *eps, abacus_nf_kind kind, const double *gm,
                       abacus_nf_sum mode, const double *kde_b, float *acc, float *rho, void *hip_stream,
                       double *acc64 = nullptr) {
    int rc = check_force_args(h, eps, kind, gm, mode, acc64 ? (const void *)acc64 : (const void *)acc);
    if (rc != ABACUS_NF_OK) return rc;
    if (kde_b) {
        if (h->n_total > 0 && !rho) return ABACUS_NF_EINVAL;
        for (int b = 0; b < h->n_boxes; b++) {
            const double bc = kde_b[b] * h->boxes[b].K / h->boxes[b].box;
            if (!std::isfinite(kde_b[b]) || !(bc >= 1e-4 && bc <= (double)h->R)) return ABACUS_NF_EINVAL;
        }
    }
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return hip_fail(hipErrorUnknown);
    if (dev != h->device) return ABACUS_NF_ESTATE;
    int *err = device_error_word(dev);
    if (!err) return ABACUS_NF_ENOMEM;
    if ((rc = ensure_work_buffers(h)) != ABACUS_NF_OK) return rc;
    hipStream_t st = (hipStream_t)hip_stream;
    if (h->n_total == 0) {   // every cell is empty: its largest |a|^2 is 0
        if (hipError_t e = launch_fill_u64(h->cell_amax, h->n_cells, 0ull, st); e != hipSuccess) return hip_fail(e);
        h->amax_valid = true;
        return ABACUS_NF_OK;
    }
    ForcesArgs a = make_args(h, kind, mode, acc, err);
    a.acc64 = acc64;
    a.rho = kde_b ? rho : nullptr;
    const int key[8] = {(int)kind, (int)mode, h->tune.sinks_per_lane, h->tune.unroll, h->tune.chunk,
                        h->tune.waves_per_cu, dev * 2 + (kde_b ? 1 : 0), h->tune.occupancy};
    if (memcmp(key, h->grid_key, sizeof(key)) != 0 || h->grid <= 0) {
        h->grid = forces_grid(h->tune, kind, mode, kde_b != nullptr, dev);
        memcpy(h->grid_key, key, sizeof(key));
    }
    a.grid = h->grid;
    mark(h, 1, false, st);
    hipError_t e = launch_set_force_boxes(eps, gm, kde_b, kind, h->boxes.data(), h->n_boxes, h->d_fbox, st);
    if (e == hipSuccess) e = build_work_list(a, st);
    mark(h, 1, true, st);
    mark(h, 2, false, st);
    if (e == hipSuccess) e = launch_forces(a, st);
    mark(h, 2, true, st);
    mark(h, 3, false, st);
    if (e == hipSuccess) e = launch_finalize(a, st);
    mark(h, 3, true, st);
    if (e != hipSuccess) return hip_fail(e);
    h->amax_valid = true;
    return ABACUS_NF_OK;
}

int abacus_nf_forces(abacus_nf_cells h, const double *eps, abacus_nf_kind kind, const double *gm,
                     abacus_nf_sum mode, float *acc, void *hip_stream) {
    return forces_impl(h, eps, kind, gm, mode, nullptr, acc, nullptr, hip_stream);
}

int abacus_nf_forces_density(abacus_nf_cells h, const double *eps, abacus_nf_kind kind, const double *gm,
                             abacus_nf_sum mode, const double *b, float *acc, float *rho, void *hip_stream) {
    if (!b) return ABACUS_NF_EINVAL;
    return forces_impl(h, eps, kind, gm, mode, b, acc, rho, hip_stream);
}

int abacus_nf_forces_f64(abacus_nf_cells h, const double *eps, abacus_nf_kind kind, const double *gm,
                         abacus_nf_sum mode, double *acc, void *hip_stream) {
    return forces_impl(h, eps, kind, gm, mode, nullptr, nullptr, nullptr, hip_stream, acc);
}

int abacus_nf_multipoles(abacus_nf_cells h, int32_t order, const double *mass, double *out, void *hip_stream) {
    if (!h || !mass) return ABACUS_NF_EINVAL;
    if (order < 0 || order > multipole_max_order()) return ABACUS_NF_EINVAL;
    if (!h->built) return ABACUS_NF_ESTATE;
    if (h->n_cells > 0 && !out) return ABACUS_NF_EINVAL;
    for (int b = 0; b < h->n_boxes; b++)
        if (!std::isfinite(mass[b])) return ABACUS_NF_EINVAL;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return hip_fail(hipErrorUnknown);
    if (dev != h->device) return ABACUS_NF_ESTATE;
    const size_t need = multipole_partial_doubles(h->n_total, order);
    if (h->mp_cap < need) {
        free_mp_buffers(h);
        if (!dalloc(h->mp_partials, need)) return ABACUS_NF_ENOMEM;
        h->mp_cap = need;
    }
    hipError_t e = launch_multipoles(h->spos, h->keys, h->cell_start, h->d_boxes, h->n_boxes, h->n_total, h->n_cells, order, mass,
                                     h->d_mass, h->mp_partials, out, dev, (hipStream_t)hip_stream);
    return e == hipSuccess ? ABACUS_NF_OK : hip_fail(e);
}

int abacus_nf_taylor_forces(abacus_nf_cells h, int32_t order, const double *taylor, float *acc, void *hip_stream) {
    if (!h) return ABACUS_NF_EINVAL;
    if (order < 0 || order > taylor_max_order()) return ABACUS_NF_EINVAL;
    if (!h->built) return ABACUS_NF_ESTATE;
    if (h->n_total > 0 && (!taylor || !acc)) return ABACUS_NF_EINVAL;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return hip_fail(hipErrorUnknown);
    if (dev != h->device) return ABACUS_NF_ESTATE;
    if (h->n_total == 0) return ABACUS_NF_OK;
    hipError_t e = launch_taylor(h->spos, h->keys, h->perm, h->d_boxes, h->n_boxes, h->n_total, h->n_cells, order,
                                 taylor, acc, dev, (hipStream_t)hip_stream);
    return e == hipSuccess ? ABACUS_NF_OK : hip_fail(e);
}

// ---------------------------------------------------------------- leapfrog time stepping (kdk.hip)

static int ensure_step_buffers(abacus_nf_cells_s *h, bool timestep) {
    if (h->scap_boxes < h->n_boxes) {
        dfree(h->d_dt);
        dfree(h->ts_min);
        h->scap_boxes = -1;
        if (!dalloc(h->d_dt, 2 * (size_t)h->n_boxes) || !dalloc(h->ts_min, timestep_min_words(h->n_boxes))) {
            free_step_buffers(h);
            return ABACUS_NF_ENOMEM;
        }
        h->scap_boxes = h->n_boxes;
    }
    if (timestep) {
        const size_t need = timestep_partial_doubles(h->n_total);
        if (h->ts_cap < need) {
            dfree(h->ts_partials);
            h->ts_cap = 0;
            if (!dalloc(h->ts_partials, need)) return ABACUS_NF_ENOMEM;
            h->ts_cap = need;
        }
    }
    return ABACUS_NF_OK;
}

static int step_checks(abacus_nf_cells h, const double *dt, int *dev) {
    if (!h || !dt) return ABACUS_NF_EINVAL;
    if (h->n_boxes < 1) return ABACUS_NF_ESTATE;
    for (int b = 0; b < h->n_boxes; b++)
        if (!std::isfinite(dt[b])) return ABACUS_NF_EINVAL;
    if (hipGetDevice(dev) != hipSuccess) return hip_fail(hipErrorUnknown);
    if (*dev != h->device) return ABACUS_NF_ESTATE;
    return ABACUS_NF_OK;
}

int abacus_nf_kick(abacus_nf_cells h, const double *dt, const float *acc, float *vel, void *hip_stream) {
    int dev = 0;
    int rc = step_checks(h, dt, &dev);
    if (rc != ABACUS_NF_OK) return rc;
    if (h->n_total > 0 && (!acc || !vel)) return ABACUS_NF_EINVAL;
    if ((rc = ensure_step_buffers(h, false)) != ABACUS_NF_OK) return rc;
    hipStream_t st = (hipStream_t)hip_stream;
    hipError_t e = upload_box_doubles(dt, h->n_boxes, h->d_dt, st);
    if (e == hipSuccess) e = launch_kick(vel, acc, h->n_total, h->d_boxes, h->n_boxes, h->d_dt, dev, st);
    return e == hipSuccess ? ABACUS_NF_OK : hip_fail(e);
}

int abacus_nf_drift(abacus_nf_cells h, const double *dt, const float *vel, float *pos, void *hip_stream) {
    int dev = 0;
    int rc = step_checks(h, dt, &dev);
    if (rc != ABACUS_NF_OK) return rc;
    if (h->n_total > 0 && (!vel || !pos)) return ABACUS_NF_EINVAL;
    if ((rc = ensure_step_buffers(h, false)) != ABACUS_NF_OK) return rc;
    hipStream_t st = (hipStream_t)hip_stream;
    double *d = h->d_dt + h->n_boxes;
    hipError_t e = upload_box_doubles(dt, h->n_boxes, d, st);
    if (e == hipSuccess) e = launch_drift(pos, vel, h->n_total, h->d_boxes, h->n_boxes, d, dev, st);
    h->built = false;   // the cells describe the old positions until the next build
    return e == hipSuccess ? ABACUS_NF_OK : hip_fail(e);
}

static int timestep_args(abacus_nf_cells h, const float *vel, const float *acc, double eta, double *dt_out) {
    if (!h || !dt_out || !std::isfinite(eta) || !(eta > 0)) return ABACUS_NF_EINVAL;
    if (!h->built) return ABACUS_NF_ESTATE;
    if (h->n_total > 0 && !vel) return ABACUS_NF_EINVAL;
    // without accelerations the maxima of a force pass since the last build are needed (none for no particles)
    if (!acc && !h->amax_valid && h->n_total > 0) return ABACUS_NF_ESTATE;
    return ABACUS_NF_OK;
}

static int timestep_checks(abacus_nf_cells h, const float *vel, const float *acc, double eta, double *dt_out,
                           int *dev) {
    const int rc = timestep_args(h, vel, acc, eta, dt_out);
    if (rc != ABACUS_NF_OK) return rc;
    if (hipGetDevice(dev) != hipSuccess) return hip_fail(hipErrorUnknown);
    if (*dev != h->device) return ABACUS_NF_ESTATE;
    return ABACUS_NF_OK;
}

// Enqueue the criterion with the given partials and per-box minima, wait, and turn the minima into steps.
// The minima are copied straight into dt_out (the caller's n_boxes doubles) and converted in place.
static int timestep_run(abacus_nf_cells h, const float *vel, const float *acc, double eta, double *dt_out,
                        double *partials, unsigned long long *dmin, hipStream_t st) {
    hipError_t e = launch_timestep(vel, acc, h->cell_amax, h->keys, h->perm, h->cell_start, h->d_boxes, h->n_boxes,
                                   h->n_total, partials, dmin, st);
    if (e != hipSuccess) return hip_fail(e);
    static_assert(sizeof(double) == sizeof(unsigned long long), "bit copies of doubles");
    if (hipMemcpyAsync(dt_out, dmin + timestep_min_offset(h->n_boxes), (size_t)h->n_boxes * sizeof(double),
                       hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return hip_fail(hipErrorUnknown);
    for (int b = 0; b < h->n_boxes; b++) {
        const double r = dt_out[b];   // the minimum sigma / |a|max (its bits were copied)
        dt_out[b] = std::isinf(r) ? r : eta * r;
    }
    return ABACUS_NF_OK;
}

int abacus_nf_timestep(abacus_nf_cells h, const float *vel, const float *acc, double eta, double *dt_out,
                       void *hip_stream) {
    int dev = 0;
    int rc = timestep_checks(h, vel, acc, eta, dt_out, &dev);
    if (rc != ABACUS_NF_OK) return rc;
    if ((rc = ensure_step_buffers(h, true)) != ABACUS_NF_OK) return rc;
    return timestep_run(h, vel, acc, eta, dt_out, h->ts_partials, h->ts_min, (hipStream_t)hip_stream);
}

}  // extern "C"

namespace anf {

int handle_boxes(abacus_nf_cells h) { return h ? h->n_boxes : 0; }

int timestep_arguments(abacus_nf_cells h, const float *vel, const float *acc, double eta, double *dt_out) {
    return timestep_args(h, vel, acc, eta, dt_out);
}

int timestep_with_buffers(abacus_nf_cells h, const float *vel, const float *acc, double eta, double *dt_out,
                          double *partials, size_t partial_doubles, unsigned long long *dmin, size_t dmin_words,
                          void *hip_stream) {
    int dev = 0;
    int rc = timestep_checks(h, vel, acc, eta, dt_out, &dev);
    if (rc != ABACUS_NF_OK) return rc;
    if (!partials || !dmin || partial_doubles < timestep_partial_doubles(h->n_total) ||
        dmin_words < timestep_min_words(h->n_boxes))
        return ABACUS_NF_EINVAL;
    return timestep_run(h, vel, acc, eta, dt_out, partials, dmin, (hipStream_t)hip_stream);
}

}  // namespace anf

extern "C" {

int abacus_nf_reorder(abacus_nf_cells h, float *const *vec3, int32_t n_vec3, int64_t *ids, void *hip_stream) {
    if (!h || n_vec3 < 0 || n_vec3 > 64 || (n_vec3 > 0 && !vec3)) return ABACUS_NF_EINVAL;
    if (!h->built) return ABACUS_NF_ESTATE;
    if (h->n_total > 0) {
        for (int k = 0; k < n_vec3; k++) {
            if (!vec3[k]) return ABACUS_NF_EINVAL;
            for (int q = 0; q < k; q++)
                if (vec3[q] == vec3[k]) return ABACUS_NF_EINVAL;   // each array once
        }
    }
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return hip_fail(hipErrorUnknown);
    if (dev != h->device) return ABACUS_NF_ESTATE;
    if (h->n_total == 0) return ABACUS_NF_OK;
    const size_t need = (size_t)h->n_total * 12;
    if (h->merge_cap < need) {
        if (h->merge_tmp) hipFree(h->merge_tmp);
        h->merge_tmp = nullptr;
        h->merge_cap = 0;
        if (!dalloc_bytes(h->merge_tmp, need)) return ABACUS_NF_ENOMEM;
        h->merge_cap = need;
    }
    hipError_t e = launch_reorder(vec3, n_vec3, ids, h->perm, h->n_total, h->merge_tmp, dev, (hipStream_t)hip_stream);
    return e == hipSuccess ? ABACUS_NF_OK : hip_fail(e);
}

int abacus_nf_kdk_step(abacus_nf_cells h, const double *dt, const double *eps, abacus_nf_kind kind,
                       const double *gm, abacus_nf_sum mode, float *pos, float *vel, float *acc, void *hip_stream) {
    int dev = 0;
    int rc = step_checks(h, dt, &dev);
    if (rc != ABACUS_NF_OK) return rc;
    if (!h->built) return ABACUS_NF_ESTATE;
    if ((rc = check_force_args(h, eps, kind, gm, mode, acc)) != ABACUS_NF_OK) return rc;
    if (h->n_total > 0 && (!pos || !vel)) return ABACUS_NF_EINVAL;
    if ((rc = ensure_step_buffers(h, false)) != ABACUS_NF_OK) return rc;
    hipStream_t st = (hipStream_t)hip_stream;
    const int nb = h->n_boxes;
    std::vector<double> half((size_t)nb);
    for (int b = 0; b < nb; b++) half[b] = 0.5 * dt[b];
    double *d_half = h->d_dt, *d_full = h->d_dt + nb;
    hipError_t e = upload_box_doubles(half.data(), nb, d_half, st);
    if (e == hipSuccess) e = upload_box_doubles(dt, nb, d_full, st);
    if (e == hipSuccess) e = launch_kick(vel, acc, h->n_total, h->d_boxes, nb, d_half, dev, st);
    if (e == hipSuccess) e = launch_drift(pos, vel, h->n_total, h->d_boxes, nb, d_full, dev, st);
    if (e != hipSuccess) return hip_fail(e);
    // move the particles to their new cells, then the forces at the new positions and the second half kick
    std::vector<abacus_nf_box> boxes = h->boxes;
    abacus_nf_cells hh = h;
    h->built = false;
    if ((rc = abacus_nf_build_cells(pos, h->n_total, boxes.data(), nb, h->R, hip_stream, &hh)) != ABACUS_NF_OK)
        return rc;
    if ((rc = forces_impl(h, eps, kind, gm, mode, nullptr, acc, nullptr, hip_stream)) != ABACUS_NF_OK) return rc;
    e = launch_kick(vel, acc, h->n_total, h->d_boxes, nb, d_half, dev, st);
    return e == hipSuccess ? ABACUS_NF_OK : hip_fail(e);
}

int abacus_nf_sync(void *hip_stream) {
    hipStream_t st = (hipStream_t)hip_stream;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return hip_fail(hipErrorUnknown);
    if (hipStreamSynchronize(st) != hipSuccess) return hip_fail(hipErrorUnknown);
    int *err = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_err_mutex);
        if (dev >= 0 && dev < kMaxDevices) err = g_err[dev];
    }
    if (!err) return ABACUS_NF_OK;
    int v = 0;
    if (hipMemcpy(&v, err, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess) return hip_fail(hipErrorUnknown);
    if (v != 0) {
        if (hipMemset(err, 0, sizeof(int)) != hipSuccess) return hip_fail(hipErrorUnknown);
        return v;
    }
    return ABACUS_NF_OK;
}

int abacus_nf_free_cells(abacus_nf_cells h) {
    if (!h) return ABACUS_NF_OK;
    int rc = ABACUS_NF_OK;
    if (h->device >= 0) {
        int cur = 0;
        if (hipGetDevice(&cur) == hipSuccess && cur != h->device) hipSetDevice(h->device);
        if (hipDeviceSynchronize() != hipSuccess) rc = hip_fail(hipErrorUnknown);
        free_sort_buffers(h);
        free_work_buffers(h);
        free_mp_buffers(h);
        free_step_buffers(h);
        destroy_events(h);
        if (cur != h->device) hipSetDevice(cur);
    }
    delete h;
    return rc;
}

int abacus_nf_interactions(abacus_nf_cells h, void *hip_stream, int64_t *out) {
    if (!h || !out) return ABACUS_NF_EINVAL;
    if (!h->built) return ABACUS_NF_ESTATE;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return hip_fail(hipErrorUnknown);
    if (dev != h->device) return ABACUS_NF_ESTATE;
    int rc = ensure_work_buffers(h);
    if (rc != ABACUS_NF_OK) return rc;
    hipStream_t st = (hipStream_t)hip_stream;
    ForcesArgs a = make_args(h, ABACUS_NF_SPLINE, ABACUS_NF_SUM_FP32, nullptr, device_error_word(dev));
    hipError_t e = launch_count_interactions(a, st);
    if (e != hipSuccess) return hip_fail(e);
    unsigned long long v = 0;
    if (hipMemcpyAsync(&v, &h->ws->interactions, sizeof(v), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return hip_fail(hipErrorUnknown);
    *out = (int64_t)v;
    return ABACUS_NF_OK;
}

int abacus_nf_cells_size(abacus_nf_cells h, int64_t *n_total, int64_t *n_cells) {
    if (!h || !n_total || !n_cells) return ABACUS_NF_EINVAL;
    if (!h->built) return ABACUS_NF_ESTATE;
    *n_total = h->n_total;
    *n_cells = h->n_cells;
    return ABACUS_NF_OK;
}

int abacus_nf_copy_cells(abacus_nf_cells h, abacus_nf_array which, void *dst, int64_t bytes, void *hip_stream) {
    if (!h || !dst) return ABACUS_NF_EINVAL;
    if (!h->built) return ABACUS_NF_ESTATE;
    const void *src = nullptr;
    int64_t want = 0;
    switch (which) {
        case ABACUS_NF_ARRAY_PERM: src = h->perm; want = h->n_total * 4; break;
        case ABACUS_NF_ARRAY_CELL_START: src = h->cell_start; want = (h->n_cells + 1) * 4; break;
        case ABACUS_NF_ARRAY_SPOS: src = h->spos; want = h->n_total * 16; break;
        case ABACUS_NF_ARRAY_CELL_KEY: src = h->keys; want = h->n_total * 4; break;
        case ABACUS_NF_ARRAY_CELL_AMAX2:
            if (!h->amax_valid) return ABACUS_NF_ESTATE;
            src = h->cell_amax;
            want = h->n_cells * 8;
            break;
        default: return ABACUS_NF_EINVAL;
    }
    if (bytes != want) return ABACUS_NF_EINVAL;
    if (want == 0) return ABACUS_NF_OK;
    if (hipMemcpyAsync(dst, src, (size_t)want, hipMemcpyDeviceToDevice, (hipStream_t)hip_stream) != hipSuccess)
        return hip_fail(hipErrorUnknown);
    return ABACUS_NF_OK;
}

int abacus_nf_set_timing(abacus_nf_cells h, int32_t enable) {
    if (!h || h->device < 0) return ABACUS_NF_EINVAL;
    if (enable && !h->ev[0]) {
        for (int i = 0; i < 8; i++)
            if (hipEventCreate(&h->ev[i]) != hipSuccess) {
                destroy_events(h);
                return hip_fail(hipErrorUnknown);
            }
    }
    for (int i = 0; i < 4; i++) h->ev_used[i] = false;
    h->timing = enable != 0;
    return ABACUS_NF_OK;
}

int abacus_nf_last_times(abacus_nf_cells h, float ms[4]) {
    if (!h || !ms) return ABACUS_NF_EINVAL;
    for (int i = 0; i < 4; i++) {
        ms[i] = -1.f;
        if (!h->ev_used[i]) continue;
        if (hipEventSynchronize(h->ev[2 * i + 1]) != hipSuccess) return hip_fail(hipErrorUnknown);
        float t = 0.f;
        if (hipEventElapsedTime(&t, h->ev[2 * i], h->ev[2 * i + 1]) != hipSuccess) return hip_fail(hipErrorUnknown);
        ms[i] = t;
    }
    return ABACUS_NF_OK;
}

int abacus_nf_set_tuning(abacus_nf_cells h, const abacus_nf_tuning *tuning) {
    if (!h) return ABACUS_NF_EINVAL;
    abacus_nf_tuning t;
    if (!resolve_tuning(tuning, &t)) return ABACUS_NF_EINVAL;
    h->tune = t;
    return ABACUS_NF_OK;
}

int abacus_nf_get_tuning(abacus_nf_cells h, abacus_nf_tuning *tuning) {
    if (!h || !tuning) return ABACUS_NF_EINVAL;
    *tuning = h->tune;
    return ABACUS_NF_OK;
}

}  // extern "C"

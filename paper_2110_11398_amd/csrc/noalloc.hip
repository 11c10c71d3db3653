// The step-size criterion for callers that cannot allocate device memory.
//
// abacus_nf_timestep keeps its unit partials and per-box minima in buffers of
// the handle, allocated by its first call.  abacus_nf_timestep_noalloc runs
// the same kernels with those two buffers carved out of one fixed array of
// device memory, `scratch`, that the library holds on each device until the
// process ends.  In host code the array's name only stands for the device
// symbol: its device address is looked up once per device with
// hipGetSymbolAddress and kept, and only that address reaches the kernels.
#include <mutex>

#include "nf_internal.h"

namespace {

// Layout of the scratch array: the per-box minima (slots and final words for up to kNoAllocMaxBoxes boxes)
// first, then the unit partials.
constexpr int kNoAllocMaxBoxes = 4096;
constexpr int64_t kNoAllocMaxParticles = int64_t(1) << 24;
constexpr size_t kNoAllocDoubles = size_t(1) << 20;   // 8 MiB per device

static __device__ __align__(256) double scratch[kNoAllocDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
double *g_scratch_addr[kMaxDevices] = {nullptr};

// Device address of this device's copy of the scratch array (looked up on the first call on the device, with
// that device current).  Returns nullptr if the lookup fails.
double *scratch_address(int dev) {
    if (dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mutex);
    if (!g_scratch_addr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
            (void)hipGetLastError();
            return nullptr;
        }
        g_scratch_addr[dev] = static_cast<double *>(p);
    }
    return g_scratch_addr[dev];
}

}  // namespace

extern "C" int abacus_nf_timestep_noalloc(abacus_nf_cells h, const float *vel, const float *acc, double eta,
                                          double *dt_out, void *hip_stream) {
    int rc = anf::timestep_arguments(h, vel, acc, eta, dt_out);
    if (rc != ABACUS_NF_OK) return rc;
    int64_t n = 0, n_cells = 0;
    if ((rc = abacus_nf_cells_size(h, &n, &n_cells)) != ABACUS_NF_OK) return rc;
    const size_t min_words = anf::timestep_min_words(kNoAllocMaxBoxes);
    if (n > kNoAllocMaxParticles || anf::handle_boxes(h) > kNoAllocMaxBoxes ||
        anf::timestep_partial_doubles(n) > kNoAllocDoubles - min_words)
        return ABACUS_NF_ELIMIT;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        return ABACUS_NF_EDEVICE;
    }
    double *base = scratch_address(dev);
    if (!base) return ABACUS_NF_EDEVICE;
    // the minima are refilled with +inf by the criterion itself, and every partial it reads is written by the
    // same call, so nothing left by an earlier call is read
    unsigned long long *dmin = reinterpret_cast<unsigned long long *>(base);
    double *partials = base + min_words;
    return anf::timestep_with_buffers(h, vel, acc, eta, dt_out, partials, kNoAllocDoubles - min_words, dmin,
                                      min_words, hip_stream);
}

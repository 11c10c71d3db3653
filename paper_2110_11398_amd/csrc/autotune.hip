// Autotuner of the force kernel: times candidate i/j tiles, unrolls and lane
// sharing on the handle's own data and keeps the fastest.  Choices can be
// cached in a small JSON file keyed by device, kind, mode and a size class.
#include <cmath>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <sstream>
#include <string>
#include <vector>

#include "nf_internal.h"

namespace {

std::string cache_key(abacus_nf_cells h, abacus_nf_kind kind, abacus_nf_sum mode, bool kde) {
    int dev = 0;
    hipGetDevice(&dev);
    hipDeviceProp_t p;
    std::string name = "gpu";
    if (hipGetDeviceProperties(&p, dev) == hipSuccess) name = p.gcnArchName;
    for (char &c : name)
        if (c == '"' || c == '\\' || c == ':') c = '_';
    int64_t n = 0, nc = 0;
    abacus_nf_cells_size(h, &n, &nc);
    const double per_cell = nc > 0 ? (double)n / (double)nc : 0.0;
    const int size_class = n > 0 ? (int)std::floor(std::log2((double)n)) : 0;
    const int occ_class = per_cell > 0 ? (int)std::floor(std::log2(per_cell) * 2) : -99;
    std::ostringstream k;
    k << name << "|k" << (int)kind << "|m" << (int)mode << "|n" << size_class << "|o" << occ_class;
    if (kde) k << "|d";
    return k.str();
}

// The cache file is a flat JSON object:
// {"key": [sinks_per_lane, chunk, unroll, max_lanes, part_sources, occupancy], ...}
std::map<std::string, std::vector<long long>> read_cache(const char *path) {
    std::map<std::string, std::vector<long long>> m;
    std::ifstream f(path);
    if (!f) return m;
    std::stringstream ss;
    ss << f.rdbuf();
    const std::string s = ss.str();
    size_t i = 0;
    while ((i = s.find('"', i)) != std::string::npos) {
        size_t j = s.find('"', i + 1);
        if (j == std::string::npos) break;
        std::string key = s.substr(i + 1, j - i - 1);
        size_t a = s.find('[', j), b = s.find(']', j);
        if (a == std::string::npos || b == std::string::npos || b < a) break;
        std::vector<long long> v;
        std::stringstream vs(s.substr(a + 1, b - a - 1));
        std::string tok;
        while (std::getline(vs, tok, ',')) v.push_back(std::atoll(tok.c_str()));
        m[key] = v;
        i = b + 1;
    }
    return m;
}

void write_cache(const char *path, const std::map<std::string, std::vector<long long>> &m) {
    std::string tmp = std::string(path) + ".tmp";
    {
        std::ofstream f(tmp);
        if (!f) return;
        f << "{\n";
        size_t k = 0;
        for (auto &kv : m) {
            f << "  \"" << kv.first << "\": [";
            for (size_t q = 0; q < kv.second.size(); q++) f << (q ? ", " : "") << kv.second[q];
            f << "]" << (++k < m.size() ? "," : "") << "\n";
        }
        f << "}\n";
    }
    std::rename(tmp.c_str(), path);
}

}  // namespace

namespace {

// One force call of the kind being tuned: the plain force, or the force with the fused density.
int force_call(abacus_nf_cells h, const double *eps, abacus_nf_kind kind, const double *gm, abacus_nf_sum mode,
               const double *kde_b, float *acc, float *rho, void *hip_stream) {
    return kde_b ? abacus_nf_forces_density(h, eps, kind, gm, mode, kde_b, acc, rho, hip_stream)
                 : abacus_nf_forces(h, eps, kind, gm, mode, acc, hip_stream);
}

int tune(abacus_nf_cells h, const double *eps, abacus_nf_kind kind, const double *gm, abacus_nf_sum mode,
         const double *kde_b, float *acc, float *rho, void *hip_stream, int32_t reps, const char *cache_path,
         abacus_nf_tuning *out) {
    if (!h || reps < 1 || reps > 100) return ABACUS_NF_EINVAL;
    abacus_nf_tuning cur;
    int rc = abacus_nf_get_tuning(h, &cur);
    if (rc) return rc;
    const std::string key = cache_key(h, kind, mode, kde_b != nullptr);
    if (cache_path) {
        auto m = read_cache(cache_path);
        auto it = m.find(key);
        if (it != m.end() && it->second.size() == 6) {
            abacus_nf_tuning t = cur;
            t.sinks_per_lane = (int32_t)it->second[0];
            t.chunk = (int32_t)it->second[1];
            t.unroll = (int32_t)it->second[2];
            t.max_lanes = (int32_t)it->second[3];
            t.part_sources = (int32_t)it->second[4];
            t.occupancy = (int32_t)it->second[5];
            if (abacus_nf_set_tuning(h, &t) == ABACUS_NF_OK) {
                rc = force_call(h, eps, kind, gm, mode, kde_b, acc, rho, hip_stream);
                if (rc == ABACUS_NF_OK) rc = abacus_nf_sync(hip_stream);
                if (rc == ABACUS_NF_OK && out) abacus_nf_get_tuning(h, out);
                return rc;
            }
        }
    }
    hipStream_t st = (hipStream_t)hip_stream;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return ABACUS_NF_EDEVICE;
    float best = 1e30f;
    abacus_nf_tuning best_t = cur;
    // time one candidate; keeps the fastest in best / best_t
    // ABACUS_NF_AUTOTUNE_LOG=1 prints every candidate's time to stderr
    const char *log_env = getenv("ABACUS_NF_AUTOTUNE_LOG");
    const bool log_trials = log_env && log_env[0] == '1';
    // A candidate whose work list outgrows its capacity (ECAPACITY, reported and cleared by the sync) is
    // skipped; any other error ends the search.
    auto trial = [&](const abacus_nf_tuning &t) -> int {
        if (abacus_nf_set_tuning(h, &t) != ABACUS_NF_OK) return ABACUS_NF_OK;  // invalid combination: skip
        int r = force_call(h, eps, kind, gm, mode, kde_b, acc, rho, hip_stream);   // warm-up (allocates if needed)
        if (r == ABACUS_NF_OK) r = abacus_nf_sync(hip_stream);
        if (r == ABACUS_NF_ECAPACITY) return ABACUS_NF_OK;
        if (r != ABACUS_NF_OK) return r;
        hipEventRecord(e0, st);
        for (int q = 0; q < reps && r == ABACUS_NF_OK; q++)
            r = force_call(h, eps, kind, gm, mode, kde_b, acc, rho, hip_stream);
        hipEventRecord(e1, st);
        if (r == ABACUS_NF_OK) r = abacus_nf_sync(hip_stream);
        if (r == ABACUS_NF_ECAPACITY) return ABACUS_NF_OK;
        if (r != ABACUS_NF_OK) return r;
        float ms = 0.f;
        hipEventElapsedTime(&ms, e0, e1);
        if (log_trials)   // one line per candidate, so long searches show progress
            fprintf(stderr, "[abacus_nf autotune] S=%d U=%d chunk=%d max_lanes=%d occupancy=%d: %.3f ms\n",
                    t.sinks_per_lane, t.unroll, t.chunk, t.max_lanes, t.occupancy, ms / reps);
        if (ms < best) {
            best = ms;
            best_t = t;
        }
        return ABACUS_NF_OK;
    };
    // stage 1: i-tile (sinks per lane), unroll and register budget on the default j-tile
    for (int S : {1, 2, 4})
        for (int U : {1, 2, 4})
            for (int occ : {0, 6, 8}) {
                abacus_nf_tuning t = cur;
                t.sinks_per_lane = S;
                t.unroll = U;
                t.occupancy = occ;
                t.chunk = 256;
                if (rc == ABACUS_NF_OK) rc = trial(t);
            }
    // stage 2: j-tile (LDS chunk) and lane sharing around the best of stage 1
    const abacus_nf_tuning s1 = best_t;
    for (int chunk : {128, 512})
        if (rc == ABACUS_NF_OK) {
            abacus_nf_tuning t = s1;
            t.chunk = chunk;
            rc = trial(t);
        }
    const abacus_nf_tuning s2 = best_t;
    for (int ml : {4, 16})
        if (rc == ABACUS_NF_OK) {
            abacus_nf_tuning t = s2;
            t.max_lanes = ml;
            rc = trial(t);
        }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (rc != ABACUS_NF_OK) {
        abacus_nf_set_tuning(h, &cur);
        return rc;
    }
    abacus_nf_set_tuning(h, &best_t);
    rc = force_call(h, eps, kind, gm, mode, kde_b, acc, rho, hip_stream);
    if (rc == ABACUS_NF_OK) rc = abacus_nf_sync(hip_stream);
    if (rc != ABACUS_NF_OK) return rc;
    if (cache_path) {
        auto m = read_cache(cache_path);
        m[key] = {best_t.sinks_per_lane, best_t.chunk, best_t.unroll, best_t.max_lanes, best_t.part_sources,
                  best_t.occupancy};
        write_cache(cache_path, m);
    }
    if (out) abacus_nf_get_tuning(h, out);
    return ABACUS_NF_OK;
}

}  // namespace

extern "C" int abacus_nf_autotune(abacus_nf_cells h, const double *eps, abacus_nf_kind kind, const double *gm,
                                  abacus_nf_sum mode, float *acc, void *hip_stream, int32_t reps,
                                  const char *cache_path, abacus_nf_tuning *out) {
    return tune(h, eps, kind, gm, mode, nullptr, acc, nullptr, hip_stream, reps, cache_path, out);
}

extern "C" int abacus_nf_autotune_density(abacus_nf_cells h, const double *eps, abacus_nf_kind kind,
                                          const double *gm, abacus_nf_sum mode, const double *b, float *acc,
                                          float *rho, void *hip_stream, int32_t reps, const char *cache_path,
                                          abacus_nf_tuning *out) {
    if (!b) return ABACUS_NF_EINVAL;
    return tune(h, eps, kind, gm, mode, b, acc, rho, hip_stream, reps, cache_path, out);
}

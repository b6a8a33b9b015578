// Autotuner of the dedispersion tile shape.
//
// Every candidate shape computes the same exact integers; they differ only in
// LDS reuse, register pressure and occupancy.  The tuner generates a
// deterministic pseudo-random 2-bit input on the device, computes a reference
// with the default shape, and for each candidate first checks that its output
// is bit-identical to the reference (candidates that differ are rejected and
// reported, never timed), then times it with HIP events.  The fastest shape
// becomes the plan's default and is stored in a small JSON cache keyed by
// (architecture, nchans, DM-count bucket, output type).
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <sstream>
#include <string>
#include <vector>

#include "dedisp_internal.hpp"

using dd::fail;

namespace {

__global__ void fill_random_kernel(uint8_t* p, int64_t n, uint64_t seed) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    // splitmix64 of (seed, index): a counter-based generator
    uint64_t z = seed + 0x9E3779B97F4A7C15ull * static_cast<uint64_t>(i + 1);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    p[i] = static_cast<uint8_t>(z);
}

__global__ void count_mismatch_kernel(const uint8_t* a, const uint8_t* b, int64_t n,
                                      unsigned long long* bad) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n && a[i] != b[i]) atomicAdd(bad, 1ull);
}

__global__ void zero_u64_kernel(unsigned long long* p) { *p = 0ull; }

std::string arch_name(int dev) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
    std::string a = prop.gcnArchName;
    const size_t colon = a.find(':');
    return colon == std::string::npos ? a : a.substr(0, colon);
}

int ndm_bucket(int ndm) {
    int b = 1;
    while (b < ndm) b <<= 1;
    return b;
}

std::string cache_key(const dedisp_plan_s* p, int out_u16) {
    std::ostringstream k;
    k << arch_name(p->device) << ":nchans=" << p->nchans << ":ndm=" << ndm_bucket(p->ndm)
      << ":" << (out_u16 ? "u16" : "i32");
    return k.str();
}

// Cache format: {"key": [dms_per_block, groups, stage_chans, ms], ...}
std::map<std::string, std::vector<double>> read_cache(const char* path) {
    std::map<std::string, std::vector<double>> m;
    if (!path) return m;
    std::ifstream f(path);
    if (!f) return m;
    std::stringstream ss;
    ss << f.rdbuf();
    const std::string s = ss.str();
    size_t pos = 0;
    while ((pos = s.find('"', pos)) != std::string::npos) {
        const size_t end = s.find('"', pos + 1);
        if (end == std::string::npos) break;
        const std::string key = s.substr(pos + 1, end - pos - 1);
        const size_t lb = s.find('[', end);
        const size_t rb = s.find(']', end);
        if (lb == std::string::npos || rb == std::string::npos || lb > rb) break;
        std::vector<double> v;
        std::stringstream nums(s.substr(lb + 1, rb - lb - 1));
        std::string tok;
        while (std::getline(nums, tok, ',')) v.push_back(std::atof(tok.c_str()));
        if (v.size() >= 3) m[key] = v;
        pos = rb + 1;
    }
    return m;
}

bool write_cache(const char* path, const std::map<std::string, std::vector<double>>& m) {
    const std::string tmp = std::string(path) + ".tmp";
    {
        std::ofstream f(tmp);
        if (!f) return false;
        f << "{\n";
        size_t i = 0;
        for (const auto& kv : m) {
            f << "  \"" << kv.first << "\": [";
            for (size_t j = 0; j < kv.second.size(); ++j) f << (j ? ", " : "") << kv.second[j];
            f << "]" << (++i < m.size() ? "," : "") << "\n";
        }
        f << "}\n";
    }
    return std::rename(tmp.c_str(), path) == 0;
}

bool valid_shape(int nd, int g, int cs) {
    const bool nd_ok = (g == 1 && (nd == 4 || nd == 8 || nd == 16 || nd == 32)) ||
                       (g == 2 && (nd == 4 || nd == 8 || nd == 16));
    return nd_ok && cs >= 4 && cs <= 128 && cs % 4 == 0;
}

}  // namespace

namespace dd {

TileConfig default_tile_config(const dedisp_plan_s* p) {
    const int packed = p->tuned.load();
    if (packed) return TileConfig{packed >> 16, (packed >> 8) & 0xFF, packed & 0xFF};
    return TileConfig{16, 1, 8};
}

TileConfig tuned_or_default(const dedisp_plan_s* p, const char* cache_path, int out_u16) {
    const auto m = read_cache(cache_path);
    const auto it = m.find(cache_key(p, out_u16));
    if (it != m.end()) {
        const int nd = static_cast<int>(it->second[0]), g = static_cast<int>(it->second[1]),
                  cs = static_cast<int>(it->second[2]);
        if (valid_shape(nd, g, cs)) return TileConfig{nd, g, cs};
    }
    return default_tile_config(p);
}

void apply_env_cache(dedisp_plan_s* p) {
    const char* path = std::getenv("DEDISP_TUNE_CACHE");
    if (!path || !*path) return;
    const auto m = read_cache(path);
    const auto it = m.find(cache_key(p, 1));
    if (it == m.end()) return;
    const int nd = static_cast<int>(it->second[0]), g = static_cast<int>(it->second[1]),
              cs = static_cast<int>(it->second[2]);
    if (valid_shape(nd, g, cs)) p->tuned.store((nd << 16) | (g << 8) | cs);
}

}  // namespace dd

extern "C" dedisp_status dedisp_autotune(dedisp_plan p, int64_t nsamps, dedisp_out_type out_type,
                                         const char* cache_path, dedisp_tile* best_out,
                                         int32_t* n_rejected) {
    if (!p) return fail(DEDISP_ERR_INVALID_ARG, "plan is NULL");
    if (out_type != DEDISP_OUT_I32 && out_type != DEDISP_OUT_U16)
        return fail(DEDISP_ERR_INVALID_ARG, "bad out_type");
    if (nsamps <= p->max_delay) return fail(DEDISP_ERR_TOO_FEW_SAMPLES, "nsamps <= max_delay");
    const int u16 = out_type == DEDISP_OUT_U16;
    const int64_t nout = nsamps - p->max_delay;
    const int64_t in_bytes = nsamps * p->nchans / 4;
    const int64_t nwords = dd::repack_words(nsamps);
    const size_t out_bytes = static_cast<size_t>(p->ndm) * nout * (u16 ? 2 : 4);
    const size_t out_alloc = (out_bytes + 255) & ~size_t(255);
    uint8_t* in = nullptr;
    uint2* words = nullptr;
    uint8_t* ref = nullptr;
    uint8_t* cand = nullptr;
    unsigned long long* bad = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipStream_t s = nullptr;
    dedisp_status st = DEDISP_OK;
    auto cleanup = [&]() {
        if (in) (void)hipFree(in);
        if (words) (void)hipFree(words);
        if (ref) (void)hipFree(ref);
        if (cand) (void)hipFree(cand);
        if (bad) (void)hipFree(bad);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        if (s) (void)hipStreamDestroy(s);
    };
    hipError_t e = hipMalloc(&in, in_bytes);
    if (e == hipSuccess) e = hipMalloc(&words, static_cast<size_t>(p->nchans) * nwords * sizeof(uint2));
    if (e == hipSuccess) e = hipMalloc(&ref, out_alloc);
    if (e == hipSuccess) e = hipMalloc(&cand, out_alloc);
    if (e == hipSuccess) e = hipMalloc(&bad, sizeof(unsigned long long));
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (e != hipSuccess) {
        cleanup();
        return fail(e == hipErrorOutOfMemory ? DEDISP_ERR_OUT_OF_MEMORY : DEDISP_ERR_HIP,
                    "autotune setup: %s", hipGetErrorString(e));
    }
    // tables built for candidate shapes are freed again, all but the winner's
    std::vector<dd::TileConfig> had = dd::offset_table_shapes(p);
    hipLaunchKernelGGL(fill_random_kernel, dim3(static_cast<unsigned>((in_bytes + 255) / 256)), dim3(256),
                       0, s, in, in_bytes, 0x5EEDull + static_cast<uint64_t>(p->ndm));
    e = dd::launch_repack(in, nsamps, p->nchans, words, nwords, s);
    const dd::TileConfig base = dd::default_tile_config(p);
    if (e == hipSuccess)
        st = dd::launch_dedisperse(p, words, nwords, nout, ref, u16, base, s);
    if (e != hipSuccess || st != DEDISP_OK) {
        cleanup();
        return st != DEDISP_OK ? st : fail(DEDISP_ERR_HIP, "autotune: %s", hipGetErrorString(e));
    }
    const int ncand = dedisp_tile_candidates(nullptr, 0);
    std::vector<dedisp_tile> cands(ncand);
    dedisp_tile_candidates(cands.data(), ncand);
    const int64_t nbytes = static_cast<int64_t>(out_bytes);
    dd::TileConfig best = base;
    float best_ms = 1e30f;
    int rejected = 0;
    for (const dedisp_tile& t : cands) {
        const dd::TileConfig c{t.dms_per_block, t.groups, t.stage_chans};
        if (dd::tile_lds_bytes(p, c) > 160 * 1024) continue;
        if (dd::launch_dedisperse(p, words, nwords, nout, cand, u16, c, s) != DEDISP_OK) continue;
        hipLaunchKernelGGL(zero_u64_kernel, dim3(1), dim3(1), 0, s, bad);
        hipLaunchKernelGGL(count_mismatch_kernel, dim3(static_cast<unsigned>((nbytes + 255) / 256)),
                           dim3(256), 0, s, ref, cand, nbytes, bad);
        unsigned long long nbad = 0;
        e = hipMemcpyAsync(&nbad, bad, sizeof nbad, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) break;
        if (nbad) {
            ++rejected;
            continue;
        }
        std::vector<float> ms;
        for (int rep = 0; rep < 3 && e == hipSuccess; ++rep) {
            e = hipEventRecord(e0, s);
            if (dd::launch_dedisperse(p, words, nwords, nout, cand, u16, c, s) != DEDISP_OK) break;
            if (e == hipSuccess) e = hipEventRecord(e1, s);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float m = 0;
            if (e == hipSuccess) e = hipEventElapsedTime(&m, e0, e1);
            ms.push_back(m);
        }
        if (ms.size() == 3) {
            std::sort(ms.begin(), ms.end());
            if (ms[1] < best_ms) {
                best_ms = ms[1];
                best = c;
            }
        }
    }
    cleanup();
    had.push_back(best);
    dd::drop_offset_tables(p, had);
    if (e != hipSuccess) return fail(DEDISP_ERR_HIP, "autotune: %s", hipGetErrorString(e));
    p->tuned.store((best.dms_per_block << 16) | (best.groups << 8) | best.stage_chans);
    if (best_out) *best_out = dedisp_tile{best.dms_per_block, best.groups, best.stage_chans};
    if (n_rejected) *n_rejected = rejected;
    if (cache_path) {
        auto m = read_cache(cache_path);
        m[cache_key(p, u16)] = {static_cast<double>(best.dms_per_block),
                                static_cast<double>(best.groups),
                                static_cast<double>(best.stage_chans), best_ms};
        if (!write_cache(cache_path, m))
            return fail(DEDISP_ERR_INVALID_ARG, "cannot write tune cache %s", cache_path);
    }
    dd::clear_error();
    return DEDISP_OK;
}

// Triage network: C API (create / load / save, tiles, forward, training step)
// and the scoring hook of the streaming server.  Kernels are in triage.hip.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "dedisp_internal.hpp"
#include "search_internal.hpp"
#include "triage_internal.hpp"
#include "triage_kernels.hpp"

using dd::fail;

struct triage_model_s {
    tk::Net net{};
    int step = 0;
    int device = 0;
    std::mutex mu;
    uint16_t* tiles = nullptr;   // scoring scratch
    int tiles_cap = 0;
};

namespace {

constexpr char kMagic[8] = {'T', 'R', 'I', 'A', 'G', 'E', '0', '1'};

void free_acts(tk::Net& n) {
    void* ptrs[] = {n.a[0], n.a[1], n.a[2], n.a[3], n.p[0], n.p[1], n.p[2], n.p[3], n.idx[0], n.idx[1],
                    n.idx[2], n.idx[3], n.g, n.logits, n.dlogit, n.dp, n.dz, n.part, n.red, n.scores};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    for (int l = 0; l < 4; ++l) n.a[l] = n.p[l] = nullptr, n.idx[l] = nullptr;
    n.g = n.logits = n.dlogit = n.dp = n.part = n.red = n.scores = nullptr;
    n.dz = nullptr;
    n.cap = 0;
}

// Activation buffers for up to `cap` tiles.
hipError_t ensure_cap(tk::Net& n, int cap) {
    if (cap <= n.cap) return hipSuccess;
    free_acts(n);
    const int Hs[4] = {64, 32, 16, 8}, Ws[4] = {256, 128, 64, 32};
    hipError_t e = hipSuccess;
    const size_t N = static_cast<size_t>(cap);
    for (int l = 0; l < 4 && e == hipSuccess; ++l) {
        const size_t full = N * Hs[l] * Ws[l] * tk::kCH, half = full / 4;
        e = hipMalloc(&n.a[l], full * 2);
        if (e == hipSuccess) e = hipMalloc(&n.p[l], half * 2);
        if (e == hipSuccess) e = hipMalloc(&n.idx[l], half);
    }
    const size_t parts = std::max<size_t>(N * 64 / tk::kRowsPerBlock * 320,
                                          N * 32 / tk::kRowsPerBlock * 9 * tk::kCH * tk::kCH);
    if (e == hipSuccess) e = hipMalloc(&n.g, N * tk::kCH * 4);
    if (e == hipSuccess) e = hipMalloc(&n.logits, N * 4);
    if (e == hipSuccess) e = hipMalloc(&n.dlogit, N * 4);
    if (e == hipSuccess) e = hipMalloc(&n.scores, N * 4);
    if (e == hipSuccess) e = hipMalloc(&n.dp, N * 32 * 128 * tk::kCH * 4);
    if (e == hipSuccess) e = hipMalloc(&n.dz, N * 64 * 256 * tk::kCH * 2);
    if (e == hipSuccess) e = hipMalloc(&n.part, parts * 4);
    if (e == hipSuccess) e = hipMalloc(&n.red, static_cast<size_t>(tk::kRedSlices) * 9 * tk::kCH * tk::kCH * 4);
    if (e == hipSuccess) n.cap = cap;
    return e;
}

void free_model(triage_model_s* m) {
    free_acts(m->net);
    void* ptrs[] = {m->net.master, m->net.grad, m->net.m, m->net.v, m->net.w1b, m->net.wfwd, m->net.wdg,
                    m->net.loss, m->net.dtap, m->net.bad, m->tiles};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    delete m;
}

// He-normal initial weights from a counter-based generator (splitmix64 +
// Box-Muller), zero biases.
void init_params(std::vector<float>& p, uint64_t seed) {
    const tk::Offsets o = tk::param_offsets();
    uint64_t ctr = seed * 0x9E3779B97F4A7C15ull + 1;
    auto u01 = [&]() {
        uint64_t z = (ctr += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        z ^= z >> 31;
        return (static_cast<double>(z >> 11) + 0.5) / 9007199254740992.0;
    };
    auto normal = [&]() { return std::sqrt(-2.0 * std::log(u01())) * std::cos(6.283185307179586 * u01()); };
    std::fill(p.begin(), p.end(), 0.0f);
    for (int i = 0; i < 32 * 9; ++i) p[o.w[0] + i] = static_cast<float>(normal() * std::sqrt(2.0 / 9));
    for (int l = 1; l < 4; ++l)
        for (int i = 0; i < 32 * 32 * 9; ++i)
            p[o.w[l] + i] = static_cast<float>(normal() * std::sqrt(2.0 / (32 * 9)));
    for (int i = 0; i < 32; ++i) p[o.wf + i] = static_cast<float>(normal() * std::sqrt(1.0 / 32));
}

dedisp_status upload(triage_model_s* m, const float* p, const float* mm, const float* vv) {
    DD_HIP(hipMemcpy(m->net.master, p, tk::kNumParams * 4, hipMemcpyHostToDevice));
    if (mm) DD_HIP(hipMemcpy(m->net.m, mm, tk::kNumParams * 4, hipMemcpyHostToDevice));
    else DD_HIP(hipMemset(m->net.m, 0, tk::kNumParams * 4));
    if (vv) DD_HIP(hipMemcpy(m->net.v, vv, tk::kNumParams * 4, hipMemcpyHostToDevice));
    else DD_HIP(hipMemset(m->net.v, 0, tk::kNumParams * 4));
    DD_HIP(tk::launch_derive(m->net.master, m->net.off, m->net.w1b, m->net.wfwd, m->net.wdg, nullptr));
    DD_HIP(hipDeviceSynchronize());
    return DEDISP_OK;
}

}  // namespace

extern "C" dedisp_status triage_create(const char* weights_path, uint64_t seed, triage_model* out) {
    if (!out) return fail(DEDISP_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    std::vector<float> p(tk::kNumParams), mm, vv;
    int step = 0;
    if (weights_path) {
        FILE* f = std::fopen(weights_path, "rb");
        if (!f) return fail(DEDISP_ERR_INVALID_ARG, "cannot open triage weights %s", weights_path);
        char magic[8];
        int32_t n = 0, st = 0;
        bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, kMagic, 8) == 0 &&
                  std::fread(&n, 4, 1, f) == 1 && n == tk::kNumParams && std::fread(&st, 4, 1, f) == 1;
        mm.resize(tk::kNumParams);
        vv.resize(tk::kNumParams);
        ok = ok && std::fread(p.data(), 4, tk::kNumParams, f) == static_cast<size_t>(tk::kNumParams) &&
             std::fread(mm.data(), 4, tk::kNumParams, f) == static_cast<size_t>(tk::kNumParams) &&
             std::fread(vv.data(), 4, tk::kNumParams, f) == static_cast<size_t>(tk::kNumParams);
        std::fclose(f);
        if (!ok) return fail(DEDISP_ERR_INVALID_ARG, "%s is not a triage model of this version", weights_path);
        for (float x : p)
            if (!std::isfinite(x)) return fail(DEDISP_ERR_INVALID_ARG, "%s holds non-finite weights", weights_path);
        step = st;
    } else {
        init_params(p, seed);
    }
    triage_model_s* m = new (std::nothrow) triage_model_s;
    if (!m) return fail(DEDISP_ERR_OUT_OF_MEMORY, "host allocation failed");
    m->net.off = tk::param_offsets();
    m->step = step;
    hipError_t e = hipGetDevice(&m->device);
    const size_t per = 32 * 9 * 32;
    if (e == hipSuccess) e = hipMalloc(&m->net.master, tk::kNumParams * 4);
    if (e == hipSuccess) e = hipMalloc(&m->net.grad, tk::kNumParams * 4);
    if (e == hipSuccess) e = hipMalloc(&m->net.m, tk::kNumParams * 4);
    if (e == hipSuccess) e = hipMalloc(&m->net.v, tk::kNumParams * 4);
    if (e == hipSuccess) e = hipMalloc(&m->net.w1b, 32 * 9 * 2);
    if (e == hipSuccess) e = hipMalloc(&m->net.wfwd, 3 * per * 2);
    if (e == hipSuccess) e = hipMalloc(&m->net.wdg, 3 * per * 2);
    if (e == hipSuccess) e = hipMalloc(&m->net.loss, 4);
    if (e == hipSuccess) e = hipMalloc(&m->net.dtap, 9 * 32 * 32 * 4);
    if (e == hipSuccess) e = hipMalloc(&m->net.bad, 4);
    if (e != hipSuccess) {
        free_model(m);
        return fail(DEDISP_ERR_OUT_OF_MEMORY, "triage model allocation: %s", hipGetErrorString(e));
    }
    dedisp_status st = upload(m, p.data(), mm.empty() ? nullptr : mm.data(), vv.empty() ? nullptr : vv.data());
    if (st != DEDISP_OK) {
        free_model(m);
        return st;
    }
    *out = m;
    dd::clear_error();
    return DEDISP_OK;
}

extern "C" dedisp_status triage_destroy(triage_model m) {
    if (!m) return fail(DEDISP_ERR_INVALID_ARG, "model is NULL");
    (void)hipDeviceSynchronize();
    free_model(m);
    return DEDISP_OK;
}

extern "C" dedisp_status triage_set_params(triage_model m, const float* host, int32_t n) {
    if (!m || !host || n != tk::kNumParams) return fail(DEDISP_ERR_INVALID_ARG, "need %d parameters", tk::kNumParams);
    std::lock_guard<std::mutex> g(m->mu);
    m->step = 0;
    return upload(m, host, nullptr, nullptr);
}

extern "C" dedisp_status triage_get_params(triage_model m, float* host, float* grads, int32_t n) {
    if (!m || n != tk::kNumParams) return fail(DEDISP_ERR_INVALID_ARG, "need %d parameters", tk::kNumParams);
    std::lock_guard<std::mutex> g(m->mu);
    DD_HIP(hipDeviceSynchronize());
    if (host) DD_HIP(hipMemcpy(host, m->net.master, n * 4, hipMemcpyDeviceToHost));
    if (grads) DD_HIP(hipMemcpy(grads, m->net.grad, n * 4, hipMemcpyDeviceToHost));
    return DEDISP_OK;
}

extern "C" int32_t triage_num_params(void) { return tk::kNumParams; }

extern "C" dedisp_status triage_forward(triage_model m, const uint16_t* tiles_bf16, int32_t n,
                                        float* logits, float* scores, dedisp_stream stream) {
    if (!m || !tiles_bf16 || n < 1) return fail(DEDISP_ERR_INVALID_ARG, "bad forward arguments");
    std::lock_guard<std::mutex> g(m->mu);
    DD_HIP(ensure_cap(m->net, n));
    DD_HIP(tk::launch_forward(m->net, tiles_bf16, n, stream));
    if (logits) DD_HIP(hipMemcpyAsync(logits, m->net.logits, n * 4, hipMemcpyDeviceToDevice, stream));
    if (scores) DD_HIP(tk::launch_sigmoid(m->net.logits, n, scores, stream));
    return DEDISP_OK;
}

extern "C" dedisp_status triage_score(triage_model m, const uint16_t* tiles_bf16, int32_t n,
                                      float* scores, dedisp_stream stream) {
    if (!scores) return fail(DEDISP_ERR_INVALID_ARG, "NULL scores");
    return triage_forward(m, tiles_bf16, n, nullptr, scores, stream);
}

extern "C" dedisp_status triage_forward_backward(triage_model m, const uint16_t* tiles_bf16,
                                                 const float* labels, int32_t n, float* loss,
                                                 dedisp_stream stream) {
    if (!m || !tiles_bf16 || !labels || n < 1) return fail(DEDISP_ERR_INVALID_ARG, "bad arguments");
    std::lock_guard<std::mutex> g(m->mu);
    DD_HIP(ensure_cap(m->net, n));
    DD_HIP(tk::launch_forward(m->net, tiles_bf16, n, stream));
    DD_HIP(tk::launch_backward(m->net, tiles_bf16, labels, n, stream));
    if (loss) {
        DD_HIP(hipMemcpyAsync(loss, m->net.loss, 4, hipMemcpyDeviceToHost, stream));
        DD_HIP(hipStreamSynchronize(stream));
    }
    return DEDISP_OK;
}

extern "C" dedisp_status triage_train_step(triage_model m, const uint16_t* tiles_bf16, const float* labels,
                                           int32_t n, float lr, float* loss, dedisp_stream stream) {
    if (!(lr > 0.0f) || !std::isfinite(lr)) return fail(DEDISP_ERR_INVALID_ARG, "lr must be > 0");
    dedisp_status st = triage_forward_backward(m, tiles_bf16, labels, n, loss, stream);
    if (st != DEDISP_OK) return st;
    std::lock_guard<std::mutex> g(m->mu);
    m->step++;
    DD_HIP(tk::launch_adam(m->net, lr, m->step, stream));
    DD_HIP(tk::launch_derive(m->net.master, m->net.off, m->net.w1b, m->net.wfwd, m->net.wdg, stream));
    return DEDISP_OK;
}

extern "C" dedisp_status triage_save(triage_model m, const char* path) {
    if (!m || !path) return fail(DEDISP_ERR_INVALID_ARG, "NULL argument");
    std::lock_guard<std::mutex> g(m->mu);
    std::vector<float> p(tk::kNumParams), mm(tk::kNumParams), vv(tk::kNumParams);
    DD_HIP(hipDeviceSynchronize());
    DD_HIP(hipMemcpy(p.data(), m->net.master, tk::kNumParams * 4, hipMemcpyDeviceToHost));
    DD_HIP(hipMemcpy(mm.data(), m->net.m, tk::kNumParams * 4, hipMemcpyDeviceToHost));
    DD_HIP(hipMemcpy(vv.data(), m->net.v, tk::kNumParams * 4, hipMemcpyDeviceToHost));
    const std::string tmp = std::string(path) + ".tmp";
    FILE* f = std::fopen(tmp.c_str(), "wb");
    if (!f) return fail(DEDISP_ERR_INVALID_ARG, "cannot write %s", path);
    const int32_t n = tk::kNumParams, st = m->step;
    bool ok = std::fwrite(kMagic, 1, 8, f) == 8 && std::fwrite(&n, 4, 1, f) == 1 && std::fwrite(&st, 4, 1, f) == 1 &&
              std::fwrite(p.data(), 4, n, f) == static_cast<size_t>(n) &&
              std::fwrite(mm.data(), 4, n, f) == static_cast<size_t>(n) &&
              std::fwrite(vv.data(), 4, n, f) == static_cast<size_t>(n);
    ok = (std::fclose(f) == 0) && ok;
    if (!ok || std::rename(tmp.c_str(), path) != 0) return fail(DEDISP_ERR_INVALID_ARG, "cannot write %s", path);
    return DEDISP_OK;
}

extern "C" dedisp_status triage_tiles(const void* series_u16, int32_t ndm, int64_t nout,
                                      const int32_t* widths, int32_t nwidths, const void* peaks_workspace,
                                      const dedisp_event* events, int32_t n_events, uint16_t* tiles_out,
                                      dedisp_stream stream) {
    if (!series_u16 || !peaks_workspace || (n_events > 0 && (!events || !tiles_out)) || ndm < 1)
        return fail(DEDISP_ERR_INVALID_ARG, "NULL argument");
    dd::Widths W;
    dedisp_status st = dd::check_widths_public(widths, nwidths, nout, &W);
    if (st != DEDISP_OK) return st;
    const dd::PeaksLayout lay = dd::peaks_layout(ndm, nout, W);
    const dd::PeaksWs ws = dd::peaks_ws(const_cast<void*>(peaks_workspace), lay);
    tk::TileWidths tw{};
    for (int i = 0; i < W.n; ++i) tw.w[i] = W.w[i];
    tw.n = W.n;
    DD_HIP(tk::launch_tiles(static_cast<const uint16_t*>(series_u16), ndm, nout, lay.nbx, tw, events, n_events,
                            ws.s1, ws.sqrt_d, tiles_out, stream));
    return DEDISP_OK;
}

namespace dd {

dedisp_status triage_score_events(triage_model m, const void* series_u16, const void* pk_ws, int ndm,
                                  int64_t nout, const Widths& W, const dedisp_event* d_events, int64_t n,
                                  std::vector<float>* scores, hipStream_t s) {
    scores->assign(static_cast<size_t>(n), 0.0f);
    if (!m) return fail(DEDISP_ERR_INVALID_ARG, "no model");
    if (n == 0) return DEDISP_OK;
    std::vector<int32_t> w(W.w, W.w + W.n);
    for (int64_t b0 = 0; b0 < n; b0 += 1024) {
        const int nb = static_cast<int>(std::min<int64_t>(1024, n - b0));
        {
            std::lock_guard<std::mutex> g(m->mu);
            if (m->tiles_cap < nb) {
                if (m->tiles) (void)hipFree(m->tiles);
                m->tiles = nullptr;
                m->tiles_cap = 0;
                DD_HIP(hipMalloc(&m->tiles, static_cast<size_t>(1024) * 64 * 256 * 2));
                m->tiles_cap = 1024;
            }
        }
        dedisp_status st = triage_tiles(series_u16, ndm, nout, w.data(), W.n, pk_ws, d_events + b0, nb, m->tiles, s);
        if (st != DEDISP_OK) return st;
        st = triage_forward(m, m->tiles, nb, nullptr, nullptr, s);
        if (st != DEDISP_OK) return st;
        {
            std::lock_guard<std::mutex> g(m->mu);
            DD_HIP(tk::launch_sigmoid(m->net.logits, nb, m->net.scores, s));
            DD_HIP(hipMemcpyAsync(scores->data() + b0, m->net.scores, nb * 4, hipMemcpyDeviceToHost, s));
            DD_HIP(hipStreamSynchronize(s));
        }
    }
    return DEDISP_OK;
}

}  // namespace dd

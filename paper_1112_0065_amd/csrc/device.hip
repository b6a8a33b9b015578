// Device description and a shader-clock probe, for reporting measured rates
// against the chip's peaks (compute units x lanes x clock).
//
// dedisp_device_info reads hipGetDeviceProperties.  dedisp_clock_probe loads
// every SIMD with dependent integer work for a given wall time and reads, in
// each wave, the shader clock counter (s_memtime) and the constant-rate
// real-time counter (s_memrealtime) at its start and end: their ratio is the
// clock the shader ran at under full vector load, which is what a VALU-bound
// kernel sees (the published peak assumes the 2.4 GHz maximum).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "dedisp_internal.hpp"

using dd::fail;

namespace {

constexpr int kProbeThreads = 256;
constexpr int kProbeMaxIter = 1 << 24;   // every wave leaves after this many rounds at most

__global__ __launch_bounds__(kProbeThreads) void clock_probe_kernel(uint64_t wall_ticks,
                                                                    unsigned long long* __restrict__ out,
                                                                    uint32_t seed) {
    const uint64_t w0 = wall_clock64();
    const uint64_t c0 = clock64();
    uint32_t a = seed + threadIdx.x, b = a ^ 0x9E3779B9u, c = a * 3u + 1u, d = a + 7u;
    uint64_t w1 = w0;
    for (int it = 0; it < kProbeMaxIter; ++it) {
#pragma unroll
        for (int k = 0; k < 64; ++k) {
            a = a * 1664525u + b;
            b = b * 22695477u + c;
            c = c * 1103515245u + d;
            d = d * 134775813u + a;
        }
        w1 = wall_clock64();
        if (w1 - w0 >= wall_ticks) break;
    }
    const uint64_t c1 = clock64();
    if ((threadIdx.x & 63) == 0) {
        const int wave = blockIdx.x * (kProbeThreads / 64) + (threadIdx.x >> 6);
        out[2 * wave] = c1 - c0;
        out[2 * wave + 1] = w1 - w0;
    }
    if ((a ^ b ^ c ^ d) == 0x12345678u) out[0] = 0;   // keeps the chains live
}

}  // namespace

extern "C" dedisp_status dedisp_device_info(dedisp_device_props* out) {
    if (!out) return fail(DEDISP_ERR_INVALID_ARG, "NULL argument");
    int dev = 0;
    DD_HIP(hipGetDevice(&dev));
    hipDeviceProp_t p;
    DD_HIP(hipGetDeviceProperties(&p, dev));
    int wall_khz = 0;
    DD_HIP(hipDeviceGetAttribute(&wall_khz, hipDeviceAttributeWallClockRate, dev));
    std::memset(out, 0, sizeof *out);
    out->device = dev;
    out->compute_units = p.multiProcessorCount;
    out->max_clock_khz = p.clockRate;
    out->memory_clock_khz = p.memoryClockRate;
    out->memory_bus_bits = p.memoryBusWidth;
    out->l2_bytes = p.l2CacheSize;
    out->lds_bytes_per_cu = static_cast<int64_t>(p.maxSharedMemoryPerMultiProcessor);
    out->total_memory_bytes = static_cast<int64_t>(p.totalGlobalMem);
    out->wall_clock_khz = wall_khz;
    std::strncpy(out->arch, p.gcnArchName, sizeof out->arch - 1);
    std::strncpy(out->name, p.name, sizeof out->name - 1);
    return DEDISP_OK;
}

extern "C" dedisp_status dedisp_clock_probe(int32_t wall_us, double* shader_ghz) {
    if (!shader_ghz || wall_us < 100 || wall_us > 2000000)
        return fail(DEDISP_ERR_INVALID_ARG, "wall_us must be in [100, 2e6] and shader_ghz non-NULL");
    dedisp_device_props props;
    dedisp_status st = dedisp_device_info(&props);
    if (st != DEDISP_OK) return st;
    if (props.wall_clock_khz <= 0) return fail(DEDISP_ERR_UNSUPPORTED, "no wall-clock rate");
    const int blocks = props.compute_units * 8;            // 8 waves per SIMD
    const int waves = blocks * (kProbeThreads / 64);
    unsigned long long* d = nullptr;
    DD_HIP(hipMalloc(&d, static_cast<size_t>(waves) * 2 * sizeof(unsigned long long)));
    const uint64_t ticks = static_cast<uint64_t>(wall_us) * props.wall_clock_khz / 1000;
    hipLaunchKernelGGL(clock_probe_kernel, dim3(blocks), dim3(kProbeThreads), 0, nullptr, ticks, d, 1u);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipDeviceSynchronize();
    std::vector<unsigned long long> h(static_cast<size_t>(waves) * 2);
    if (e == hipSuccess) e = hipMemcpy(h.data(), d, h.size() * sizeof h[0], hipMemcpyDeviceToHost);
    (void)hipFree(d);
    if (e != hipSuccess) return fail(DEDISP_ERR_HIP, "clock probe: %s", hipGetErrorString(e));
    std::vector<double> ghz;
    for (int w = 0; w < waves; ++w) {
        const double dt = static_cast<double>(h[2 * w + 1]) / (props.wall_clock_khz * 1e3);
        if (dt > 0) ghz.push_back(static_cast<double>(h[2 * w]) / dt * 1e-9);
    }
    if (ghz.empty()) return fail(DEDISP_ERR_HIP, "clock probe recorded nothing");
    std::nth_element(ghz.begin(), ghz.begin() + ghz.size() / 2, ghz.end());
    *shader_ghz = ghz[ghz.size() / 2];
    return DEDISP_OK;
}

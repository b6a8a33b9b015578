// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdarg>
#include <cstdint>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/dedisp.h"

namespace dd {

// Record the message for dedisp_last_error() and return the status.
dedisp_status fail(dedisp_status st, const char* fmt, ...);
void clear_error();

#define DD_HIP(expr)                                                          \
    do {                                                                      \
        hipError_t e_ = (expr);                                               \
        if (e_ != hipSuccess)                                                 \
            return ::dd::fail(DEDISP_ERR_HIP, "%s failed: %s", #expr,         \
                              hipGetErrorString(e_));                         \
    } while (0)

// Number of bit-slice levels the accumulator needs for sums <= 3*nchans.
inline int levels_for(int nchans) { return 3 * nchans <= 4095 ? 12 : 16; }

// Tile shapes of the dedispersion kernel.
struct TileConfig {
    int dms_per_block;   // DM trials sharing one LDS tile (multiple of the waves)
    int groups;          // 32-sample groups per lane (time tile = 2048*groups)
    int stage_chans;     // channels per LDS stage (multiple of 4)
};

// Everything the dedispersion kernel needs about one beam.
struct BeamArgs {
    const uint2* words;      // channel-major bit-plane copy [nchans][nwords]
    int64_t nwords;
    int nchans;
    int ndm;
    int64_t nout;
    const int32_t* delays;   // [ndm][nchans]
    const uint32_t* offs;    // [ndm][nchans] LDS read offsets for the tile shape
    const int32_t* skew;     // per DM block, for the tile's block size
    void* out;               // [ndm][nout]
    int n_dm_blocks;
    int tile_words;          // T/32 + 1 of the launch's tile shape
    int pitch;               // 16-byte quads per LDS row: tile_words - 1 + the largest block skew
    int dm_group;            // DM blocks per group of the work-item order
    int64_t item_begin;      // first work item of this beam in a batch
    int64_t n_items;         // time tiles x DM blocks
};

// Words (uint2 = one 32-sample lo/hi bit-plane pair) per channel in the
// channel-major copy of the input.
inline int64_t repack_words(int64_t nsamps) { return 2 * ((nsamps + 63) / 64) + 2; }

}  // namespace dd

struct dedisp_plan_s {
    int32_t nchans = 0;
    int32_t ndm = 0;
    double f_top = 0, df = 0, tsamp = 0;
    std::vector<double> dm_list;
    std::vector<int32_t> delays;      // host copy [ndm][nchans]
    int64_t max_delay = 0;
    int32_t* d_delays = nullptr;      // device copy [ndm][nchans]
    int device = 0;
    // Per DM-block skew (in 32-sample words) for each supported block size.
    static constexpr int kNumDmBlock = 4;          // 4, 8, 16, 32 DMs
    int32_t* d_skew[kNumDmBlock] = {nullptr, nullptr, nullptr, nullptr};
    int32_t skew_max[kNumDmBlock] = {0, 0, 0, 0};
    // Tile shape chosen by the autotuner (dms << 16 | groups << 8 | stage), 0 = default.
    std::atomic<int> tuned{0};
    // Per tile shape: the LDS read offset and funnel shift of every (trial,
    // channel), built on first use of the shape (dd::offset_table).
    struct OffsetTable {
        int dms, groups, stage;
        uint32_t* d;
    };
    mutable std::mutex tab_mu;
    mutable std::vector<OffsetTable> tabs;
};

namespace dd {

inline int dm_block_index(int dms_per_block) {
    switch (dms_per_block) {
        case 4: return 0;
        case 8: return 1;
        case 16: return 2;
        case 32: return 3;
        default: return -1;
    }
}

// Kernel launchers (asynchronous; return hipError_t of the launch).
hipError_t launch_repack(const uint8_t* in, int64_t nsamps, int nchans, uint2* words,
                         int64_t nwords, hipStream_t s, const uint8_t* mask = nullptr,
                         int64_t mask_n = 0);
dedisp_status launch_dedisperse(const dedisp_plan_s* p, const uint2* words,
                                int64_t nwords, int64_t nout, void* out, int out_u16,
                                const TileConfig& cfg, hipStream_t s);
TileConfig default_tile_config(const dedisp_plan_s* p);
void apply_env_cache(dedisp_plan_s* p);
BeamArgs beam_args(const dedisp_plan_s* p, const uint2* words, int64_t nwords, int64_t nout,
                   void* out, const TileConfig& cfg);
size_t tile_lds_bytes(const dedisp_plan_s* p, const TileConfig& cfg);
int tile_pitch(const dedisp_plan_s* p, const TileConfig& cfg);
// Device table of the tile shape, [ndm][nchans] entries
//     ((c mod CS) * pitch + (delay[d][c] >> 5) - (delay[d_lo][c] >> 5)) * 16 << 5
//   | (delay[d][c] & 31)
// with d_lo the block's first trial and pitch = 64*G + (largest block skew)
// quads per row: the byte offset, in an LDS stage buffer, of the quad (the
// 16-byte copy of two consecutive words) the trial reads first for channel
// c, and the shift within it.  Built (synchronously: hipMalloc + hipMemcpy) on first use of the
// shape; `build` false only looks it up.  Returns nullptr on failure.
const uint32_t* offset_table(const dedisp_plan_s* p, const TileConfig& cfg, bool build,
                             dedisp_status* st = nullptr);
// Free the tables of every shape not in `keep`; the shapes that have one.
void drop_offset_tables(const dedisp_plan_s* p, const std::vector<TileConfig>& keep);
std::vector<TileConfig> offset_table_shapes(const dedisp_plan_s* p);
// Persistent multi-beam launch (beams: device array, item ranges filled).
hipError_t launch_dedisperse_persistent(const BeamArgs* d_beams, int nbeams, int64_t total,
                                        int nl, int out_u16, const TileConfig& cfg, size_t lds,
                                        unsigned long long* d_counters, int nq, int grid,
                                        hipStream_t s);
// One beam (or one streamed window) of a multi-item run.
struct MultiItem {
    const dedisp_plan_s* plan;
    const uint8_t* in;      // device, packed 2-bit input
    int64_t nsamps;
    void* words;            // device, bit-plane workspace
    void* out;              // device series [ndm][nsamps - max_delay]
    void* pk_ws;            // device find_peaks workspace
    dedisp_event* events;   // device, capacity records
    int64_t capacity;
    int64_t* h_total;       // pinned host: number of events found
    const uint8_t* mask;    // device coincidence mask of samples [0, mask_n), or NULL
    int64_t mask_n;
    void* flat;             // device [ndm][nout - 2R] baseline-removed series, or NULL
};
// Persistent grid size for this shape on `device` (multiple of nq; 0 on error).
int batch_grid(int nl, int out_u16, const TileConfig& cfg, size_t lds, int device, int nq);
// Resident blocks per CU of the persistent kernel for this shape (0 on error).
int persistent_blocks_per_cu(int nl, int out_u16, const TileConfig& cfg, size_t lds);

}  // namespace dd

// Internal declarations of the boxcar / sigma-cut / peak-finding stage.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "../../include/dedisp.h"
#include "dedisp_internal.hpp"

namespace dd {

constexpr int kMaxWidths = 32;

// Boxcar widths, passed by value to kernels.
struct Widths {
    int32_t w[kMaxWidths];
    int32_t n;
};

// Device workspace of find_peaks (all arrays live in one caller buffer).
struct PeaksWs {
    uint64_t* part_s1;     // [nw][ndm][nseg]
    uint64_t* part_s2lo;   // [nw][ndm][nseg]
    uint64_t* part_s2hi;   // [nw][ndm][nseg]
    uint32_t* part_max;    // [nw][ndm][nseg] largest B of the segment
    uint64_t* s1;          // [nw][ndm]
    uint64_t* s2lo;        // [nw][ndm]
    uint64_t* s2hi;        // [nw][ndm]
    int64_t* thr;          // [nw][ndm], -1: no events (D == 0)
    uint32_t* thr32;       // [nw][ndm], 0xFFFFFFFF: nothing can pass
    double* sqrt_d;        // [nw][ndm]
    uint32_t* counts;      // [nw][ndm][nseg] run starts
    int64_t* offs;         // [nw][ndm][nseg] exclusive scan of counts
    int64_t* chunk_tot;    // scan scratch
    int64_t* total;        // total number of events
    uint32_t* list;        // [ndm * nseg] (DM, segment)s to count (d * nseg + seg)
    uint32_t* list2;       // [ndm * nseg] (DM, segment)s with events
    uint32_t* nlist;       // [2] lengths of list and list2
};

struct PeaksLayout {
    int64_t nbx;
    int L;
    int nseg;
    int64_t nseries;
    int64_t ncounts;
    int nchunks;
    size_t o_part_s1, o_part_s2lo, o_part_s2hi, o_part_max, o_s1, o_s2lo, o_s2hi, o_thr, o_thr32, o_sqrt_d,
        o_counts, o_offs, o_chunk, o_total, o_list, o_list2, o_nlist;
    size_t bytes;
};

int segment_length(int w_max);
PeaksLayout peaks_layout(int ndm, int64_t nout, const Widths& W);
PeaksWs peaks_ws(void* base, const PeaksLayout& lay);

// Exclusive scan of n uint32 counts into int64 offsets (total in *total);
// chunk_tot needs scan_chunk_count(n) entries.
hipError_t launch_scan_u32(const uint32_t* counts, int64_t n, int64_t* offs, int64_t* chunk_tot,
                           int64_t* total, hipStream_t s);
int64_t scan_chunk_count(int64_t n);
size_t cluster_workspace_bytes(int64_t n, int32_t ndm, int32_t nwidths);
hipError_t launch_cluster(const dedisp_event* ev, int64_t n, int32_t ndm, const int32_t* widths,
                          int32_t nwidths, int32_t dm_radius, int32_t width_radius, int64_t time_tol,
                          dedisp_cluster* out, int64_t capacity, int32_t* labels, void* ws,
                          const int64_t** result, hipStream_t s);
hipError_t launch_baseline(const void* in, int in_u16, int ndm, int64_t nout, int radius,
                           int offset, void* out, int out_u16, hipStream_t s);
hipError_t launch_boxcar(const void* in, int in_u16, int ndm, int64_t nout, const Widths& W,
                         int dm_first, int dm_count, int32_t* out, hipStream_t s);
// Stats, thresholds, run-start counts and their scan (total in ws.total).
hipError_t launch_peaks_count(const void* in, int in_u16, int ndm, int64_t nout, const Widths& W,
                              const PeaksLayout& lay, const PeaksWs& ws, uint32_t kmant, int kexp2,
                              hipStream_t s);
hipError_t launch_peaks_write(const void* in, int in_u16, int ndm, int64_t nout, const Widths& W,
                              const PeaksLayout& lay, const PeaksWs& ws, dedisp_event* events,
                              int64_t capacity, hipStream_t s);

// Shared by the batch and the streaming server: see batch.cpp.  Items with a
// mask read flagged samples as the mean level; items with a `flat` buffer get
// baseline removal of radius bl_radius (offset bl_offset) before the search.
hipError_t launch_multi(const MultiItem* items, int n, const Widths& W, uint32_t kmant, int kexp2,
                        int out_u16, const TileConfig& cfg, int nl, size_t lds, int grid, int nq,
                        BeamArgs* h_beams, BeamArgs* d_beams, unsigned long long* d_counters,
                        hipStream_t s, int bl_radius = 0, int bl_offset = 0);
// Coincidence mask (coincidence.hip): asynchronous, the number of flagged
// samples left on the device (rfi_mask_count); workspace rfi_mask_ws_bytes.
size_t rfi_mask_ws_bytes(int nbeams, int64_t nsamps);
hipError_t launch_rfi_mask(const uint8_t* const* ins, int nbeams, int nchans, int64_t nsamps,
                           uint32_t kmant, int kexp2, int min_beams, uint8_t* mask, void* workspace,
                           hipStream_t stream);
const unsigned long long* rfi_mask_count(const void* workspace, int nbeams, int64_t nsamps);
hipError_t launch_rfi_apply(uint8_t* const* beams, int nbeams, int nchans, int64_t nsamps,
                            const uint8_t* mask, hipStream_t stream);
dedisp_status split_threshold_public(float k, uint32_t* kmant, int* kexp2);
dedisp_status check_widths_public(const int32_t* widths, int32_t nwidths, int64_t nout, Widths* W);
TileConfig tuned_or_default(const dedisp_plan_s* p, const char* cache_path, int out_u16);

}  // namespace dd

// Streaming server: real-time search of every beam's chunks as they arrive.
//
// The paper's goal is detection in real time, as the telescope observes
// (sections 1 and 3), with the 13 beams of the multibeam receiver (section 1)
// arriving continuously at about 4 MB/s each.  This engine takes each beam's
// chunks of C samples, keeps on the device the last H = max_delay + w_max - 1
// input samples of every beam (the overlap the next chunk's dedispersion and
// widest boxcar need), admits chunks into device slots sized against an HBM
// budget, and continuously batches: whenever slots are free, every queued
// chunk of any beam joins the next persistent launch, while the copies of
// that batch overlap the compute of the previous one (separate streams).
//
// Chunk k >= 1 of a beam (contiguous after chunk k-1) is searched over the
// window of absolute samples [kC - H, (k+1)C), giving exactly C boxcar start
// positions; the first chunk of a beam (or the first after a gap) has no
// overlap and gives C - H positions.  The concatenated integer results equal
// the one-shot result.  Statistics of the sigma-cut are those of each chunk.
//
// Threads: callers (submit / poll), one scheduler (assembles and launches
// batches), one completion thread (waits for a batch, copies events back,
// records latency, frees slots).
#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "dedisp_internal.hpp"
#include "search_internal.hpp"
#include "triage_internal.hpp"

using dd::fail;

extern "C" int64_t dedisp_percentile_ns(const int64_t* sorted, int64_t n, double q);
extern "C" int32_t dedisp_serve_admission(size_t budget, size_t resident, size_t slot_bytes);

namespace {

int64_t now_ns() {
    return std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

struct Slot {
    uint8_t* window = nullptr;    // packed input window (H + C samples max)
    void* words = nullptr;        // bit-plane workspace
    void* out = nullptr;          // uint16 series
    void* pk_ws = nullptr;        // find_peaks workspace
    dedisp_event* d_events = nullptr;
    dedisp_event* d_cand = nullptr;     // the events triage scores (after selection)
    void* cl_ws = nullptr;              // clustering workspace (when enabled)
    dedisp_cluster* d_clusters = nullptr;
    void* flat = nullptr;               // baseline-removed series (when that stage is on)
    bool busy = false;
};

struct Job {
    int beam = 0;
    int64_t seq = 0;
    int64_t arrival_ns = 0;
    int32_t flags = 0;
    int host_buf = -1;       // index of the pinned staging buffer
    int slot = -1;
    int64_t t_abs0 = 0;      // absolute sample index of the window start
    int64_t nsamps = 0;      // window length
    bool overlap = false;
    int64_t* h_total = nullptr;
};

struct Batch {
    std::vector<Job> jobs;
    hipEvent_t done = nullptr;
    int ring = 0;
};

struct Result {
    dedisp_chunk_result r;
    std::vector<dedisp_event> events;
    std::vector<float> scores;
    std::vector<dedisp_cluster> clusters;
};

}  // namespace

struct dedisp_server_s {
    std::vector<dedisp_plan> plans;
    int nbeams = 0;
    int64_t C = 0;
    int64_t H = 0;                 // max over beams of max_delay + w_max - 1
    std::vector<int64_t> Hb;       // per beam
    int nchans = 0;
    dd::Widths W{};
    uint32_t kmant = 0;
    int kexp2 = 0;
    dd::TileConfig cfg{};
    int nl = 12;
    size_t lds = 0;
    int grid = 0;
    int nq = 8;
    int64_t capacity = 1 << 16;
    triage_model model = nullptr;
    float triage_thresh = 0.5f;
    double deadline_ns = 0;
    int64_t ndm_max = 0;
    size_t budget = 0;             // HBM budget of the overlaps and chunk slots
    bool draining = false;         // destroy: release incomplete rounds
    // optional stages (dedisp_serve_set_stages)
    int bl_radius = 0;             // baseline removal radius, 0 = off
    int rfi_min = 0;               // coincidence mask: min beams, 0 = off
    uint32_t rfi_kmant = 0;
    int rfi_kexp2 = 0;
    void* rfi_ws = nullptr;        // mask workspace and mask of one round (copy stream)
    uint8_t* d_mask = nullptr;
    // clustering of each chunk's events (dedisp_serve_set_clustering)
    bool cluster_on = false;
    int32_t cl_dm_radius = 0, cl_width_radius = 0;
    int64_t cl_time_tol = 0;

    // device
    std::vector<uint8_t*> overlap;       // per beam, H_b samples of packed input
    std::vector<Slot> slots;
    static constexpr int kRing = 4;      // batches in flight
    dd::BeamArgs* h_beams[kRing] = {};
    dd::BeamArgs* d_beams[kRing] = {};
    unsigned long long* d_counters = nullptr;
    int64_t* h_totals = nullptr;         // pinned, one per slot
    std::vector<uint8_t*> host_bufs;     // pinned chunk staging
    std::vector<bool> host_busy;
    hipStream_t copy_s = nullptr, comp_s = nullptr, done_s = nullptr;

    // per-beam stream state (scheduler side)
    std::vector<int64_t> next_seq;       // expected next sequence number (submit side)
    int submitting = 0;                  // submits between admission and the pending queue
    std::vector<bool> have_overlap;

    // queues
    std::mutex mu;
    std::condition_variable cv_sched, cv_done, cv_poll;
    std::deque<Job> pending;
    std::deque<Batch> inflight;
    std::deque<Result> results;
    std::vector<Result> last_polled;
    bool stop = false;
    int ring_next = 0;
    int ring_used = 0;
    dedisp_status async_error = DEDISP_OK;
    std::string async_msg;

    // statistics
    std::vector<int64_t> latencies;
    int64_t batches = 0, batched_chunks = 0, misses = 0, max_batch = 0;

    std::thread sched, compl_;
};

namespace {

void set_async_error(dedisp_server_s* s, dedisp_status st, const char* what, hipError_t e) {
    std::lock_guard<std::mutex> g(s->mu);
    if (s->async_error == DEDISP_OK) {
        s->async_error = st;
        s->async_msg = std::string(what) + ": " + hipGetErrorString(e);
    }
    s->stop = true;
    s->cv_poll.notify_all();
    s->cv_sched.notify_all();
    s->cv_done.notify_all();
}

// Assemble one job's window on copy_s: [overlap | chunk], then save the new
// overlap.  Runs in the scheduler thread in per-beam sequence order.
hipError_t assemble(dedisp_server_s* s, Job& j) {
    const int64_t bpc = s->nchans / 4;   // bytes per sample
    const int64_t Hb = s->Hb[j.beam];
    Slot& sl = s->slots[j.slot];
    hipError_t e = hipSuccess;
    int64_t off = 0;
    if (j.overlap) {
        e = hipMemcpyAsync(sl.window, s->overlap[j.beam], Hb * bpc, hipMemcpyDeviceToDevice, s->copy_s);
        off = Hb;
    }
    if (e == hipSuccess)
        e = hipMemcpyAsync(sl.window + off * bpc, s->host_bufs[j.host_buf], s->C * bpc,
                           hipMemcpyHostToDevice, s->copy_s);
    j.nsamps = off + s->C;
    return e;
}

// Save the window's last H_b samples as the beam's next overlap.
hipError_t save_overlap(dedisp_server_s* s, const Job& j) {
    const int64_t bpc = s->nchans / 4;
    const int64_t Hb = s->Hb[j.beam];
    return hipMemcpyAsync(s->overlap[j.beam], s->slots[j.slot].window + (j.nsamps - Hb) * bpc,
                          Hb * bpc, hipMemcpyDeviceToDevice, s->copy_s);
}

// Coincidence mask of one round: the new C samples of every job's window
// (the overlaps were masked with their own round), applied in place before
// the overlaps are saved.  On copy_s, in stream order with the assembly.
hipError_t mask_round(dedisp_server_s* s, const std::vector<Job>& round) {
    const int64_t bpc = s->nchans / 4;
    std::vector<uint8_t*> news;
    for (const Job& j : round) news.push_back(s->slots[j.slot].window + (j.nsamps - s->C) * bpc);
    const int n = static_cast<int>(news.size());
    std::vector<const uint8_t*> cnews(news.begin(), news.end());
    hipError_t e = dd::launch_rfi_mask(cnews.data(), n, s->nchans, s->C, s->rfi_kmant, s->rfi_kexp2,
                                       s->rfi_min, s->d_mask, s->rfi_ws, s->copy_s);
    if (e == hipSuccess) e = dd::launch_rfi_apply(news.data(), n, s->nchans, s->C, s->d_mask, s->copy_s);
    return e;
}

// With the coincidence mask: is the round of the lowest pending sequence
// number k ready -- every beam has submitted k or a later chunk (a beam that
// skipped k sits the round out) and a slot is free for each of the round's
// chunks?  Called with s->mu held.
bool round_ready(const dedisp_server_s* s, int64_t* k_out) {
    int64_t k = INT64_MAX;
    for (const Job& j : s->pending) k = std::min(k, j.seq);
    if (k == INT64_MAX) return false;
    if (s->submitting > 0 && !s->draining) return false;   // a chunk of the round may be on its way
    for (int64_t q : s->next_seq)
        if (q <= k && !s->draining) return false;
    size_t nfree = 0, nk = 0;
    for (const Slot& sl : s->slots) nfree += sl.busy ? 0 : 1;
    for (const Job& j : s->pending) nk += j.seq == k ? 1 : 0;
    if (k_out) *k_out = k;
    return nk <= nfree;
}

void scheduler(dedisp_server_s* s) {
    hipSetDevice(s->plans[0]->device);
    hipEvent_t copied = nullptr;
    if (hipEventCreateWithFlags(&copied, hipEventDisableTiming) != hipSuccess) return;
    for (;;) {
        std::vector<Job> take;
        int ring = 0;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv_sched.wait(lk, [&] {
                if (s->stop) return true;
                if (s->pending.empty() || s->ring_used >= dedisp_server_s::kRing) return false;
                if (s->rfi_min) return round_ready(s, nullptr);
                for (const Slot& sl : s->slots)
                    if (!sl.busy) return true;
                return false;
            });
            if (s->stop) break;
            // with the coincidence mask, whole rounds only: the pending
            // chunks of the lowest sequence number, once every beam has
            // submitted it (or passed it: a gap), and only when a slot is
            // free for each of them
            std::vector<Job> round;
            if (s->rfi_min) {
                int64_t k = 0;
                round_ready(s, &k);
                for (auto it = s->pending.begin(); it != s->pending.end();) {
                    if (it->seq == k) {
                        round.push_back(*it);
                        it = s->pending.erase(it);
                    } else {
                        ++it;
                    }
                }
            }
            // every pending chunk (any beam, in arrival order) while slots
            // last, or the round
            for (size_t i = 0; i < s->slots.size() && (s->rfi_min ? !round.empty() : !s->pending.empty()); ++i) {
                if (s->slots[i].busy) continue;
                Job j;
                if (s->rfi_min) {
                    j = round.front();
                    round.erase(round.begin());
                } else {
                    j = s->pending.front();
                    s->pending.pop_front();
                }
                s->slots[i].busy = true;
                j.slot = static_cast<int>(i);
                j.h_total = &s->h_totals[i];
                // overlap bookkeeping in sequence order
                j.overlap = s->have_overlap[j.beam] && !(j.flags & DEDISP_CHUNK_GAP);
                j.t_abs0 = j.seq * s->C - (j.overlap ? s->Hb[j.beam] : 0);
                s->have_overlap[j.beam] = true;
                take.push_back(j);
            }
            ring = s->ring_next;
            s->ring_next = (s->ring_next + 1) % dedisp_server_s::kRing;
            s->ring_used++;
        }
        hipError_t e = hipSuccess;
        if (s->rfi_min) {
            // one chunk per beam: every window, then the round's mask, then
            // the (masked) overlaps
            for (Job& j : take)
                if (e == hipSuccess) e = assemble(s, j);
            if (e == hipSuccess) e = mask_round(s, take);
            for (Job& j : take)
                if (e == hipSuccess) e = save_overlap(s, j);
        } else {
            // a batch may hold consecutive chunks of one beam: each window
            // takes the overlap its predecessor just saved
            for (Job& j : take) {
                if (e == hipSuccess) e = assemble(s, j);
                if (e == hipSuccess) e = save_overlap(s, j);
            }
        }
        if (e == hipSuccess) e = hipEventRecord(copied, s->copy_s);
        if (e == hipSuccess) e = hipStreamWaitEvent(s->comp_s, copied, 0);
        std::vector<dd::MultiItem> items(take.size());
        for (size_t i = 0; i < take.size(); ++i) {
            const Slot& sl = s->slots[take[i].slot];
            items[i] = dd::MultiItem{s->plans[take[i].beam], sl.window, take[i].nsamps, sl.words, sl.out,
                                     sl.pk_ws, sl.d_events, s->capacity, take[i].h_total, nullptr, 0,
                                     s->bl_radius ? sl.flat : nullptr};
        }
        if (e == hipSuccess)
            e = dd::launch_multi(items.data(), static_cast<int>(items.size()), s->W, s->kmant, s->kexp2, 1,
                                 s->cfg, s->nl, s->lds, s->grid, s->nq, s->h_beams[ring],
                                 s->d_beams[ring], s->d_counters, s->comp_s, s->bl_radius,
                                 3 * s->nchans);
        Batch b;
        b.jobs = std::move(take);
        b.ring = ring;
        if (e == hipSuccess) e = hipEventCreateWithFlags(&b.done, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventRecord(b.done, s->comp_s);
        if (e != hipSuccess) {
            set_async_error(s, DEDISP_ERR_HIP, "batch launch", e);
            break;
        }
        {
            std::lock_guard<std::mutex> g(s->mu);
            s->inflight.push_back(std::move(b));
            s->batches++;
            s->batched_chunks += static_cast<int64_t>(s->inflight.back().jobs.size());
            s->max_batch = std::max<int64_t>(s->max_batch, s->inflight.back().jobs.size());
        }
        s->cv_done.notify_one();
    }
    (void)hipEventDestroy(copied);
}

void completer(dedisp_server_s* s) {
    hipSetDevice(s->plans[0]->device);
    for (;;) {
        Batch b;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv_done.wait(lk, [&] { return s->stop || !s->inflight.empty(); });
            if (s->inflight.empty()) break;   // stop requested and nothing left
            b = std::move(s->inflight.front());
            s->inflight.pop_front();
        }
        hipError_t e = hipEventSynchronize(b.done);
        (void)hipEventDestroy(b.done);
        std::vector<Result> done;
        for (Job& j : b.jobs) {
            Result r{};
            const int64_t n = e == hipSuccess ? *j.h_total : 0;
            const int64_t m = std::min(n, s->capacity);
            r.events.resize(static_cast<size_t>(m));
            if (e == hipSuccess && m > 0)
                e = hipMemcpyAsync(r.events.data(), s->slots[j.slot].d_events, m * sizeof(dedisp_event),
                                   hipMemcpyDeviceToHost, s->done_s);
            if (e == hipSuccess) e = hipStreamSynchronize(s->done_s);
            int32_t flags = j.flags;
            if (n > s->capacity) flags |= DEDISP_CHUNK_OVERFLOW;
            if (e == hipSuccess && s->cluster_on) {
                const Slot& sl = s->slots[j.slot];
                int64_t nc = 0;
                if (m > 0) {
                    const int64_t* d_result = nullptr;
                    int64_t back[2] = {0, 0};   // count, error flag
                    e = dd::launch_cluster(sl.d_events, m, s->plans[j.beam]->ndm, s->W.w, s->W.n,
                                           s->cl_dm_radius, s->cl_width_radius, s->cl_time_tol,
                                           sl.d_clusters, s->capacity, nullptr, sl.cl_ws, &d_result,
                                           s->done_s);
                    if (e == hipSuccess)
                        e = hipMemcpyAsync(back, d_result, sizeof back, hipMemcpyDeviceToHost, s->done_s);
                    if (e == hipSuccess) e = hipStreamSynchronize(s->done_s);
                    // find_peaks output always passes the input checks; a
                    // failed check leaves the chunk unclustered
                    nc = static_cast<uint32_t>(back[1]) ? -1 : std::min(back[0], s->capacity);
                    if (e == hipSuccess && nc > 0) {
                        r.clusters.resize(static_cast<size_t>(nc));
                        e = hipMemcpyAsync(r.clusters.data(), sl.d_clusters, nc * sizeof(dedisp_cluster),
                                           hipMemcpyDeviceToHost, s->done_s);
                        if (e == hipSuccess) e = hipStreamSynchronize(s->done_s);
                    }
                }
                if (nc >= 0) {
                    flags |= DEDISP_CHUNK_CLUSTERED;
                    r.r.n_clusters = nc;
                }
            }
            if (e == hipSuccess && s->model) {
                // the network scores candidates: the events per-width
                // non-maximum suppression keeps (the selection it was trained
                // on); suppressed events get no score (-1)
                const dedisp_plan_s* p = s->plans[j.beam];
                const int64_t nout = j.nsamps - p->max_delay - 2 * static_cast<int64_t>(s->bl_radius);
                const Slot& sl = s->slots[j.slot];
                const void* series = s->bl_radius ? sl.flat : sl.out;
                std::vector<int64_t> keep(static_cast<size_t>(std::max<int64_t>(m, 1)));
                int64_t nk = 0;
                dedisp_status tst = dedisp_candidates_nms(r.events.data(), m, s->W.w, s->W.n, 32, 128,
                                                          keep.data(), &nk);
                std::vector<dedisp_event> cand(static_cast<size_t>(nk));
                for (int64_t k = 0; k < nk; ++k) cand[static_cast<size_t>(k)] = r.events[static_cast<size_t>(keep[k])];
                if (tst == DEDISP_OK && nk > 0) {
                    e = hipMemcpyAsync(sl.d_cand, cand.data(), nk * sizeof(dedisp_event),
                                       hipMemcpyHostToDevice, s->done_s);
                    if (e != hipSuccess) tst = DEDISP_ERR_HIP;
                }
                std::vector<float> cs;
                if (tst == DEDISP_OK)
                    tst = dd::triage_score_events(s->model, series, sl.pk_ws, p->ndm, nout, s->W, sl.d_cand,
                                                  nk, &cs, s->done_s);
                if (tst == DEDISP_OK) {
                    r.scores.assign(static_cast<size_t>(m), -1.0f);
                    for (int64_t k = 0; k < nk; ++k) r.scores[static_cast<size_t>(keep[k])] = cs[static_cast<size_t>(k)];
                    r.r.n_candidates = nk;
                } else {
                    flags |= DEDISP_CHUNK_FALLBACK;
                }
            } else if (!s->model) {
                flags |= DEDISP_CHUNK_FALLBACK;
            }
            r.r.beam = j.beam;
            r.r.seq = j.seq;
            // with baseline removal the search covers the flattened series,
            // which starts at dedispersed sample R of the window
            r.r.t_abs0 = j.t_abs0 + s->bl_radius;
            r.r.n_bx = j.nsamps - s->plans[j.beam]->max_delay - 2 * static_cast<int64_t>(s->bl_radius) -
                       s->W.w[s->W.n - 1] + 1;
            r.r.n_events = n;
            r.r.arrival_ns = j.arrival_ns;
            r.r.done_ns = now_ns();
            if (r.r.done_ns - j.arrival_ns > s->deadline_ns) flags |= DEDISP_CHUNK_LATE;
            r.r.flags = flags;
            done.push_back(std::move(r));
        }
        if (e != hipSuccess) {
            set_async_error(s, DEDISP_ERR_HIP, "batch completion", e);
            break;
        }
        {
            std::lock_guard<std::mutex> g(s->mu);
            for (Job& j : b.jobs) {
                s->slots[j.slot].busy = false;
                s->host_busy[j.host_buf] = false;
            }
            s->ring_used--;
            for (Result& r : done) {
                s->latencies.push_back(r.r.done_ns - r.r.arrival_ns);
                if (r.r.flags & DEDISP_CHUNK_LATE) s->misses++;
                s->results.push_back(std::move(r));
            }
        }
        s->cv_sched.notify_one();
        s->cv_poll.notify_all();
    }
}

// Device and pinned buffers sized by the chunk, the stages and the budget
// (not the streams or threads).
void free_buffers(dedisp_server_s* s) {
    for (uint8_t* p : s->overlap)
        if (p) (void)hipFree(p);
    s->overlap.clear();
    for (Slot& sl : s->slots) {
        if (sl.window) (void)hipFree(sl.window);
        if (sl.words) (void)hipFree(sl.words);
        if (sl.out) (void)hipFree(sl.out);
        if (sl.pk_ws) (void)hipFree(sl.pk_ws);
        if (sl.d_events) (void)hipFree(sl.d_events);
        if (sl.d_cand) (void)hipFree(sl.d_cand);
        if (sl.cl_ws) (void)hipFree(sl.cl_ws);
        if (sl.d_clusters) (void)hipFree(sl.d_clusters);
        if (sl.flat) (void)hipFree(sl.flat);
    }
    s->slots.clear();
    for (int i = 0; i < dedisp_server_s::kRing; ++i) {
        if (s->h_beams[i]) (void)hipHostFree(s->h_beams[i]);
        if (s->d_beams[i]) (void)hipFree(s->d_beams[i]);
        s->h_beams[i] = nullptr;
        s->d_beams[i] = nullptr;
    }
    if (s->h_totals) (void)hipHostFree(s->h_totals);
    s->h_totals = nullptr;
    for (uint8_t* p : s->host_bufs)
        if (p) (void)hipHostFree(p);
    s->host_bufs.clear();
    s->host_busy.clear();
    if (s->rfi_ws) (void)hipFree(s->rfi_ws);
    if (s->d_mask) (void)hipFree(s->d_mask);
    s->rfi_ws = nullptr;
    s->d_mask = nullptr;
}

void free_server(dedisp_server_s* s) {
    free_buffers(s);
    if (s->d_counters) (void)hipFree(s->d_counters);
    if (s->copy_s) (void)hipStreamDestroy(s->copy_s);
    if (s->comp_s) (void)hipStreamDestroy(s->comp_s);
    if (s->done_s) (void)hipStreamDestroy(s->done_s);
    delete s;
}

// Bytes of one chunk slot: window, workspace, series (and its baseline-
// removed copy), search workspace, events and candidates.
size_t slot_bytes(const std::vector<dedisp_plan>& plans, int64_t C, const dd::Widths& W, int R) {
    int64_t H = 0, ndm = 0, nchans = 0;
    const int w_max = W.w[W.n - 1];
    for (const dedisp_plan_s* p : plans) {
        H = std::max<int64_t>(H, p->max_delay + w_max - 1 + 2 * static_cast<int64_t>(R));
        ndm = std::max<int64_t>(ndm, p->ndm);
        nchans = std::max<int64_t>(nchans, p->nchans);
    }
    const int64_t win = H + C;
    const int64_t nser = C + w_max - 1;              // series length the search covers
    const size_t a = static_cast<size_t>(win * nchans / 4);
    const size_t b = static_cast<size_t>(nchans) * dd::repack_words(win) * sizeof(uint2);
    const size_t c = static_cast<size_t>(ndm) * (nser + 2 * static_cast<int64_t>(R)) * 2;
    const size_t f = R ? static_cast<size_t>(ndm) * nser * 2 : 0;
    const size_t d = dd::peaks_layout(static_cast<int>(ndm), nser, W).bytes;
    const size_t e = 2 * static_cast<size_t>(1 << 16) * sizeof(dedisp_event);   // events, candidates
    return a + b + c + f + d + e;
}

// Overlaps per beam, then as many chunk slots as the budget holds; the
// coincidence mask needs one slot per beam (a round at once).
dedisp_status setup_buffers(dedisp_server_s* s) {
    const int w_max = s->W.w[s->W.n - 1];
    const int64_t R = s->bl_radius;
    s->Hb.clear();
    s->H = 0;
    for (int b = 0; b < s->nbeams; ++b) {
        s->Hb.push_back(s->plans[b]->max_delay + w_max - 1 + 2 * R);
        s->H = std::max(s->H, s->Hb.back());
    }
    if (s->C <= s->H)
        return fail(DEDISP_ERR_TOO_FEW_SAMPLES, "chunk of %lld samples <= overlap %lld",
                    static_cast<long long>(s->C), static_cast<long long>(s->H));
    if ((s->C + s->H + 16384 + w_max) * 4 >= (int64_t(1) << 31))
        return fail(DEDISP_ERR_UNSUPPORTED, "chunk of %lld samples too long",
                    static_cast<long long>(s->C));
    const int nchans = s->nchans;
    const size_t sb = slot_bytes(s->plans, s->C, s->W, s->bl_radius);
    size_t resident = 0;
    for (int b = 0; b < s->nbeams; ++b) resident += static_cast<size_t>(s->Hb[b] * nchans / 4);
    const int nslots = dedisp_serve_admission(s->budget, resident, sb);
    if (nslots < 1)
        return fail(DEDISP_ERR_OUT_OF_MEMORY,
                    "HBM budget %zu bytes below overlap (%zu) + one chunk slot (%zu)", s->budget,
                    resident, sb);
    if (s->rfi_min && nslots < s->nbeams)
        return fail(DEDISP_ERR_OUT_OF_MEMORY,
                    "the coincidence mask takes a round of %d chunks at once: the budget holds %d slots",
                    s->nbeams, nslots);
    hipError_t e = hipSuccess;
    const int64_t win = s->H + s->C;
    const int64_t nser = s->C + w_max - 1;
    s->overlap.assign(s->nbeams, nullptr);
    for (int b = 0; b < s->nbeams && e == hipSuccess; ++b)
        e = hipMalloc(&s->overlap[b], static_cast<size_t>(s->Hb[b] * nchans / 4));
    s->slots.resize(nslots);
    size_t wsb = 0;
    for (const dedisp_plan_s* p : s->plans)
        wsb = std::max(wsb, static_cast<size_t>(p->nchans) * dd::repack_words(win) * sizeof(uint2));
    const size_t cl_ws = s->cluster_on ? dd::cluster_workspace_bytes(s->capacity, static_cast<int32_t>(s->ndm_max), s->W.n) : 0;
    for (int i = 0; i < nslots && e == hipSuccess; ++i) {
        Slot& sl = s->slots[i];
        e = hipMalloc(&sl.window, static_cast<size_t>(win * nchans / 4));
        if (e == hipSuccess) e = hipMalloc(&sl.words, wsb);
        if (e == hipSuccess) e = hipMalloc(&sl.out, static_cast<size_t>(s->ndm_max) * (nser + 2 * R) * 2);
        if (e == hipSuccess && R) e = hipMalloc(&sl.flat, static_cast<size_t>(s->ndm_max) * nser * 2);
        if (e == hipSuccess)
            e = hipMalloc(&sl.pk_ws, dd::peaks_layout(static_cast<int>(s->ndm_max), nser, s->W).bytes);
        if (e == hipSuccess) e = hipMalloc(&sl.d_events, static_cast<size_t>(s->capacity) * sizeof(dedisp_event));
        if (e == hipSuccess) e = hipMalloc(&sl.d_cand, static_cast<size_t>(s->capacity) * sizeof(dedisp_event));
        if (e == hipSuccess && cl_ws) e = hipMalloc(&sl.cl_ws, cl_ws);
        if (e == hipSuccess && cl_ws)
            e = hipMalloc(&sl.d_clusters, static_cast<size_t>(s->capacity) * sizeof(dedisp_cluster));
    }
    for (int i = 0; i < dedisp_server_s::kRing && e == hipSuccess; ++i) {
        e = hipHostMalloc(&s->h_beams[i], sizeof(dd::BeamArgs) * nslots, hipHostMallocDefault);
        if (e == hipSuccess) e = hipMalloc(&s->d_beams[i], sizeof(dd::BeamArgs) * nslots);
    }
    if (e == hipSuccess) e = hipHostMalloc(&s->h_totals, sizeof(int64_t) * nslots, hipHostMallocDefault);
    const int nhost = 2 * nslots + s->nbeams;
    s->host_bufs.assign(nhost, nullptr);
    s->host_busy.assign(nhost, false);
    for (int i = 0; i < nhost && e == hipSuccess; ++i)
        e = hipHostMalloc(&s->host_bufs[i], static_cast<size_t>(s->C * nchans / 4), hipHostMallocDefault);
    if (e == hipSuccess && s->rfi_min) {
        e = hipMalloc(&s->rfi_ws, dd::rfi_mask_ws_bytes(s->nbeams, s->C));
        if (e == hipSuccess) e = hipMalloc(&s->d_mask, static_cast<size_t>(s->C));
    }
    if (e != hipSuccess)
        return fail(e == hipErrorOutOfMemory ? DEDISP_ERR_OUT_OF_MEMORY : DEDISP_ERR_HIP,
                    "server buffers: %s", hipGetErrorString(e));
    return DEDISP_OK;
}

}  // namespace

extern "C" int64_t dedisp_now_ns(void) { return now_ns(); }

extern "C" int64_t dedisp_percentile_ns(const int64_t* sorted, int64_t n, double q) {
    // nearest-rank percentile of an ascending array
    if (!sorted || n <= 0) return 0;
    int64_t k = static_cast<int64_t>(std::ceil(q * static_cast<double>(n) - 1e-9));
    k = std::max<int64_t>(1, std::min<int64_t>(k, n));
    return sorted[k - 1];
}

extern "C" int32_t dedisp_serve_admission(size_t budget, size_t resident, size_t slot_bytes) {
    if (slot_bytes == 0 || budget < resident + slot_bytes) return 0;
    return static_cast<int32_t>(std::min<size_t>(4096, (budget - resident) / slot_bytes));
}

extern "C" size_t dedisp_serve_slot_bytes(const dedisp_plan* plans, int32_t nbeams,
                                          int64_t chunk_nsamps, const int32_t* widths,
                                          int32_t nwidths) {
    if (!plans || nbeams < 1 || chunk_nsamps < 1 || !widths || nwidths < 1) return 0;
    for (int b = 0; b < nbeams; ++b)
        if (!plans[b]) return 0;
    dd::Widths W;
    if (dd::check_widths_public(widths, nwidths, chunk_nsamps + widths[nwidths - 1] - 1, &W) != DEDISP_OK)
        return 0;
    return slot_bytes(std::vector<dedisp_plan>(plans, plans + nbeams), chunk_nsamps, W, 0);
}

extern "C" dedisp_status dedisp_serve_create(const dedisp_plan* plans, int32_t nbeams,
                                             int64_t chunk_nsamps, const int32_t* widths,
                                             int32_t nwidths, float snr_thresh,
                                             size_t hbm_budget_bytes, triage_model model,
                                             dedisp_server* out) {
    if (!out || !plans || nbeams < 1 || nbeams > 1024 || chunk_nsamps < 64)
        return fail(DEDISP_ERR_INVALID_ARG, "need plans, 1..1024 beams, chunk of >= 64 samples");
    *out = nullptr;
    const int nchans = plans[0] ? plans[0]->nchans : 0;
    for (int b = 0; b < nbeams; ++b) {
        if (!plans[b]) return fail(DEDISP_ERR_INVALID_ARG, "plan %d is NULL", b);
        if (plans[b]->nchans != nchans)
            return fail(DEDISP_ERR_UNSUPPORTED, "all beams need the same channel count");
        if (plans[b]->device != plans[0]->device)
            return fail(DEDISP_ERR_INVALID_ARG, "all plans must be on one device");
    }
    dd::Widths W;
    dedisp_status st = dd::check_widths_public(widths, nwidths, INT64_C(1) << 20, &W);
    if (st != DEDISP_OK) return st;
    uint32_t km;
    int ke;
    st = dd::split_threshold_public(snr_thresh, &km, &ke);
    if (st != DEDISP_OK) return st;
    dedisp_server_s* s = new (std::nothrow) dedisp_server_s;
    if (!s) return fail(DEDISP_ERR_OUT_OF_MEMORY, "host allocation failed");
    s->plans.assign(plans, plans + nbeams);
    s->nbeams = nbeams;
    s->C = chunk_nsamps;
    s->nchans = nchans;
    s->W = W;
    s->kmant = km;
    s->kexp2 = ke;
    s->model = model;
    s->budget = hbm_budget_bytes;
    s->deadline_ns = static_cast<double>(s->C) * plans[0]->tsamp * 1e9;
    s->nl = dd::levels_for(nchans);
    s->cfg = dd::default_tile_config(plans[0]);
    for (int b = 0; b < nbeams; ++b) s->lds = std::max(s->lds, dd::tile_lds_bytes(plans[b], s->cfg));
    s->grid = dd::batch_grid(s->nl, 1, s->cfg, s->lds, plans[0]->device, s->nq);
    if (s->lds > 160 * 1024 || s->grid < 1) {
        delete s;
        return fail(DEDISP_ERR_UNSUPPORTED, "tile shape does not fit (LDS %zu bytes)", s->lds);
    }
    for (int b = 0; b < nbeams; ++b) {
        dedisp_status st = DEDISP_OK;
        if (!dd::offset_table(plans[b], s->cfg, true, &st)) {
            delete s;
            return st;
        }
    }
    int64_t ndm_max = 0;
    for (int b = 0; b < nbeams; ++b) ndm_max = std::max<int64_t>(ndm_max, plans[b]->ndm);
    s->ndm_max = ndm_max;
    // HBM admission: resident overlaps first, then as many chunk slots as fit.
    st = setup_buffers(s);
    if (st != DEDISP_OK) {
        free_server(s);
        return st;
    }
    hipError_t e = hipMalloc(&s->d_counters, sizeof(unsigned long long) * s->nq);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->copy_s, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->comp_s, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->done_s, hipStreamNonBlocking);
    if (e != hipSuccess) {
        free_server(s);
        return fail(e == hipErrorOutOfMemory ? DEDISP_ERR_OUT_OF_MEMORY : DEDISP_ERR_HIP,
                    "server setup: %s", hipGetErrorString(e));
    }
    s->next_seq.assign(nbeams, -1);
    s->have_overlap.assign(nbeams, false);
    s->sched = std::thread(scheduler, s);
    s->compl_ = std::thread(completer, s);
    *out = s;
    dd::clear_error();
    return DEDISP_OK;
}

extern "C" dedisp_status dedisp_serve_submit(dedisp_server s, int32_t beam, int64_t seq,
                                             const uint8_t* host_chunk, int64_t arrival_ns) {
    if (!s || !host_chunk || beam < 0 || beam >= s->nbeams || seq < 0)
        return fail(DEDISP_ERR_INVALID_ARG, "bad submit arguments");
    int hb = -1;
    int32_t flags = 0;
    {
        std::lock_guard<std::mutex> g(s->mu);
        if (s->async_error != DEDISP_OK) return fail(s->async_error, "%s", s->async_msg.c_str());
        const int64_t expect = s->next_seq[beam];
        if (expect >= 0 && seq < expect)
            return fail(DEDISP_ERR_INVALID_ARG, "beam %d: chunk %lld arrives after chunk %lld", beam,
                        static_cast<long long>(seq), static_cast<long long>(expect - 1));
        for (size_t i = 0; i < s->host_busy.size(); ++i)
            if (!s->host_busy[i]) {
                hb = static_cast<int>(i);
                break;
            }
        if (hb < 0) return DEDISP_ERR_BUSY;   // back-pressure: not admitted yet
        s->host_busy[hb] = true;
        if (expect >= 0 && seq > expect) flags |= DEDISP_CHUNK_GAP;
        s->next_seq[beam] = seq + 1;
        s->submitting++;
    }
    std::memcpy(s->host_bufs[hb], host_chunk, static_cast<size_t>(s->C * s->nchans / 4));
    Job j;
    j.beam = beam;
    j.seq = seq;
    j.arrival_ns = arrival_ns;
    j.flags = flags;
    j.host_buf = hb;
    {
        std::lock_guard<std::mutex> g(s->mu);
        s->pending.push_back(j);
        s->submitting--;
    }
    s->cv_sched.notify_one();
    dd::clear_error();
    return DEDISP_OK;
}

extern "C" dedisp_status dedisp_serve_poll(dedisp_server s, dedisp_chunk_result* out, int32_t cap,
                                           int32_t* n_out, int32_t timeout_ms) {
    if (!s || !n_out || (cap > 0 && !out)) return fail(DEDISP_ERR_INVALID_ARG, "bad poll arguments");
    *n_out = 0;
    std::unique_lock<std::mutex> lk(s->mu);
    if (timeout_ms > 0 && s->results.empty() && s->async_error == DEDISP_OK)
        s->cv_poll.wait_for(lk, std::chrono::milliseconds(timeout_ms),
                            [&] { return !s->results.empty() || s->async_error != DEDISP_OK; });
    if (s->async_error != DEDISP_OK) return fail(s->async_error, "%s", s->async_msg.c_str());
    s->last_polled.clear();
    while (!s->results.empty() && static_cast<int32_t>(s->last_polled.size()) < cap) {
        s->last_polled.push_back(std::move(s->results.front()));
        s->results.pop_front();
    }
    for (size_t i = 0; i < s->last_polled.size(); ++i) {
        Result& r = s->last_polled[i];
        r.r.events = r.events.empty() ? nullptr : r.events.data();
        r.r.scores = r.scores.empty() ? nullptr : r.scores.data();
        r.r.clusters = r.clusters.empty() ? nullptr : r.clusters.data();
        out[i] = r.r;
    }
    *n_out = static_cast<int32_t>(s->last_polled.size());
    return DEDISP_OK;
}

extern "C" dedisp_status dedisp_serve_stats(dedisp_server s, dedisp_serve_stats_t* st) {
    if (!s || !st) return fail(DEDISP_ERR_INVALID_ARG, "NULL argument");
    std::lock_guard<std::mutex> g(s->mu);
    std::vector<int64_t> l = s->latencies;
    std::sort(l.begin(), l.end());
    auto pct = [&](double q) { return dedisp_percentile_ns(l.data(), static_cast<int64_t>(l.size()), q); };
    st->chunks_done = static_cast<int64_t>(l.size());
    st->p50_ns = pct(0.50);
    st->p99_ns = pct(0.99);
    st->max_ns = l.empty() ? 0 : l.back();
    st->deadline_misses = s->misses;
    st->batches = s->batches;
    st->max_batch = s->max_batch;
    st->mean_batch = s->batches ? static_cast<double>(s->batched_chunks) / s->batches : 0.0;
    st->slots = static_cast<int32_t>(s->slots.size());
    st->deadline_ns = static_cast<int64_t>(s->deadline_ns);
    return DEDISP_OK;
}

extern "C" dedisp_status dedisp_serve_set_clustering(dedisp_server s, int32_t dm_radius,
                                                     int32_t width_radius, int64_t time_tol) {
    if (!s) return fail(DEDISP_ERR_INVALID_ARG, "server is NULL");
    if (dm_radius < 0 || dm_radius > 65535 || width_radius < 0 || width_radius > 31 ||
        time_tol < 0 || time_tol > (int64_t(1) << 40))
        return fail(DEDISP_ERR_INVALID_ARG, "radius or tolerance out of range");
    std::lock_guard<std::mutex> g(s->mu);
    for (int64_t q : s->next_seq)
        if (q >= 0) return fail(DEDISP_ERR_BUSY, "clustering must be set before the first submit");
    if (!s->cluster_on) {
        const size_t ws = dd::cluster_workspace_bytes(s->capacity, static_cast<int32_t>(s->ndm_max),
                                                      s->W.n);
        hipError_t e = hipSuccess;
        for (Slot& sl : s->slots) {
            if (e == hipSuccess) e = hipMalloc(&sl.cl_ws, ws);
            if (e == hipSuccess)
                e = hipMalloc(&sl.d_clusters, static_cast<size_t>(s->capacity) * sizeof(dedisp_cluster));
        }
        if (e != hipSuccess) {
            for (Slot& sl : s->slots) {
                if (sl.cl_ws) (void)hipFree(sl.cl_ws);
                if (sl.d_clusters) (void)hipFree(sl.d_clusters);
                sl.cl_ws = nullptr;
                sl.d_clusters = nullptr;
            }
            return fail(e == hipErrorOutOfMemory ? DEDISP_ERR_OUT_OF_MEMORY : DEDISP_ERR_HIP,
                        "clustering buffers: %s", hipGetErrorString(e));
        }
    }
    s->cl_dm_radius = dm_radius;
    s->cl_width_radius = width_radius;
    s->cl_time_tol = time_tol;
    s->cluster_on = true;
    dd::clear_error();
    return DEDISP_OK;
}

extern "C" dedisp_status dedisp_serve_set_stages(dedisp_server s, float rfi_k_sigma,
                                                 int32_t rfi_min_beams, int32_t baseline_radius) {
    if (!s) return fail(DEDISP_ERR_INVALID_ARG, "server is NULL");
    uint32_t km = 0;
    int ke = 0;
    if (rfi_k_sigma != 0.0f) {
        const dedisp_status st = dd::split_threshold_public(rfi_k_sigma, &km, &ke);
        if (st != DEDISP_OK) return st;
        if (rfi_min_beams < 1 || rfi_min_beams > s->nbeams || s->nbeams > 64)
            return fail(DEDISP_ERR_INVALID_ARG, "min_beams %d outside [1, %d] (at most 64 beams)",
                        rfi_min_beams, s->nbeams);
    }
    if (baseline_radius < 0 || baseline_radius > 8192)
        return fail(DEDISP_ERR_INVALID_ARG, "baseline radius %d outside [0, 8192]", baseline_radius);
    if (baseline_radius > 0 && 6 * s->nchans > 65535)
        return fail(DEDISP_ERR_UNSUPPORTED, "uint16 baseline output needs 6 nchans <= 65535");
    std::lock_guard<std::mutex> g(s->mu);
    for (int64_t q : s->next_seq)
        if (q >= 0) return fail(DEDISP_ERR_BUSY, "stages must be set before the first submit");
    // nothing is in flight: size the buffers for the new stages
    const int old_r = s->bl_radius, old_m = s->rfi_min;
    const uint32_t old_km = s->rfi_kmant;
    const int old_ke = s->rfi_kexp2;
    free_buffers(s);
    s->bl_radius = baseline_radius;
    s->rfi_min = rfi_k_sigma != 0.0f ? rfi_min_beams : 0;
    s->rfi_kmant = km;
    s->rfi_kexp2 = ke;
    dedisp_status st = setup_buffers(s);
    if (st != DEDISP_OK) {
        const std::string msg = dedisp_last_error();
        free_buffers(s);
        s->bl_radius = old_r;
        s->rfi_min = old_m;
        s->rfi_kmant = old_km;
        s->rfi_kexp2 = old_ke;
        if (setup_buffers(s) != DEDISP_OK) {
            s->async_error = DEDISP_ERR_OUT_OF_MEMORY;
            s->async_msg = "server buffers could not be restored";
        }
        return fail(st, "%s", msg.c_str());
    }
    dd::clear_error();
    return DEDISP_OK;
}

extern "C" dedisp_status dedisp_serve_destroy(dedisp_server s) {
    if (!s) return fail(DEDISP_ERR_INVALID_ARG, "server is NULL");
    {
        // let queued work finish before stopping (rounds of the coincidence
        // mask that some beam never completed go as they are)
        std::unique_lock<std::mutex> lk(s->mu);
        s->draining = true;
        s->cv_sched.notify_all();
        s->cv_poll.wait_for(lk, std::chrono::seconds(600), [&] {
            return s->async_error != DEDISP_OK || (s->pending.empty() && s->inflight.empty() && s->ring_used == 0);
        });
        s->stop = true;
    }
    s->cv_sched.notify_all();
    s->cv_done.notify_all();
    if (s->sched.joinable()) s->sched.join();
    if (s->compl_.joinable()) s->compl_.join();
    (void)hipDeviceSynchronize();
    free_server(s);
    return DEDISP_OK;
}

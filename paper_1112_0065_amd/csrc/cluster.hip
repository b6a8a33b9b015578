// Event clustering across DM trials and boxcar widths.
//
// Section 2.3 ends the search by gathering the contiguous above-cut samples of
// one series into events.  A dispersed pulse crosses the cut in many
// neighbouring trials and widths, so one pulse gives many events; this stage
// merges them into candidates.  The merging rule (the paper names only the
// per-series gathering) is friends of friends:
//
//   * event e covers samples [t_start, t_end + W - 1], W = widths[width_idx];
//   * a and b are friends when |dm_a - dm_b| <= dm_radius,
//     |width_idx_a - width_idx_b| <= width_radius and their spans are at most
//     time_tol samples apart;
//   * a cluster is a connected component of that relation, numbered in the
//     order of its lowest-index member; its representative is the member of
//     largest snr, ties to the lower index.
//
// Design.  The events arrive in (width_idx, dm_idx, t_start) order with
// disjoint, increasing runs inside a series, so the friends of an event in a
// neighbouring series form one contiguous index range, found by a binary
// search on t_end.  A table of series starts comes from one pass over the
// list.  Components are built by lock-free union-find on a parent array: a
// root is only ever hooked under a smaller root (one compare-and-swap), and
// finds halve paths with plain word stores that only ever point a node at one
// of its ancestors.  Every node's parent is therefore smaller than the node,
// and each finished component's root is its lowest member whatever order the
// threads ran in -- the result is deterministic.  Member counts, index and
// time bounds and the representative (the largest (snr, -index) key) are
// integer atomics into the root's slot; a scan over the roots numbers the
// clusters.  The work is a handful of dependent loads per event, so the
// stage is bound by memory latency, not bandwidth.
#include <algorithm>
#include <climits>

#include "dedisp_internal.hpp"
#include "search_internal.hpp"

namespace {

constexpr int kKThreads = 256;

struct ClusterParams {
    const dedisp_event* ev;
    int64_t n;
    int32_t ndm;
    int32_t nwidths;
    int32_t dm_radius;
    int32_t width_radius;
    int64_t time_tol;
    int32_t widths[dd::kMaxWidths];
};

__device__ __forceinline__ int atomic_ld(const int32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void atomic_st(int32_t* p, int32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// A node that was a root when seen.  Parents only ever decrease, so the walk
// ends; a stale halving store still points the node at one of its ancestors.
__device__ int find_root(int32_t* parent, int32_t x) {
    int32_t p = atomic_ld(parent + x);
    while (p != x) {
        const int32_t g = atomic_ld(parent + p);
        if (g == p) return p;
        atomic_st(parent + x, g);   // x is not a root, so no hook can race with this store
        x = g;
        p = atomic_ld(parent + x);
    }
    return x;
}

// An ancestor of x through wavefront-scope (cached) loads.  A cached parent
// value may be old, but every value a parent slot ever held is an ancestor of
// its node for good (trees only merge), so the result is always an ancestor
// and equal results prove two nodes joined.  The walk ends because parents
// decrease.
__device__ int32_t find_cached(const int32_t* parent, int32_t x) {
    int32_t p = __hip_atomic_load(parent + x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
    while (p != x) {
        x = p;
        p = __hip_atomic_load(parent + x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
    }
    return x;
}

__device__ void unite(int32_t* parent, int32_t a, int32_t b) {
    while (true) {
        a = find_root(parent, a);
        b = find_root(parent, b);
        if (a == b) return;
        if (a > b) {
            const int32_t t = a;
            a = b;
            b = t;
        }
        int32_t expect = b;
        if (__hip_atomic_compare_exchange_strong(parent + b, &expect, a, __ATOMIC_RELAXED,
                                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
            return;
        // b was hooked meanwhile: retry from the new roots
    }
}

__device__ __forceinline__ bool event_ok(const dedisp_event& e, const ClusterParams& P) {
    return e.width_idx >= 0 && e.width_idx < P.nwidths && e.dm_idx >= 0 && e.dm_idx < P.ndm &&
           e.t_start >= 0 && e.t_end >= e.t_start && e.t_end < (int64_t(1) << 62) &&
           !__builtin_isnan(e.snr);
}

// Totally ordered key of (snr, -index): larger snr first, then lower index.
__device__ __forceinline__ uint64_t rep_key(float snr, int64_t i) {
    uint32_t u = __float_as_uint(snr);
    if (u == 0x80000000u) u = 0;                      // -0 ranks as +0
    u = (u & 0x80000000u) ? ~u : (u | 0x80000000u);
    return (static_cast<uint64_t>(u) << 32) | (0xFFFFFFFFu - static_cast<uint32_t>(i));
}

__global__ void cluster_init_kernel(uint32_t* err) { *err = 0; }

// Series starts: seg[k] = first event with series key >= k, k = w * ndm + d,
// for k in [0, nwidths * ndm]; thread i (0 <= i <= n) fills the keys between
// event i - 1's and its own.  Also checks the input order and fields, and
// starts every event as its own root.
__global__ __launch_bounds__(kKThreads) void cluster_seg_kernel(ClusterParams P,
                                                                int32_t* __restrict__ seg,
                                                                int32_t* __restrict__ parent,
                                                                uint32_t* __restrict__ err) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kKThreads + threadIdx.x;
    if (i > P.n) return;
    if (i < P.n) parent[i] = static_cast<int32_t>(i);
    const int64_t K = static_cast<int64_t>(P.nwidths) * P.ndm;
    int64_t kprev = -1, kcur = K;
    bool bad = false;
    if (i > 0) {
        const dedisp_event a = P.ev[i - 1];
        if (event_ok(a, P)) kprev = static_cast<int64_t>(a.width_idx) * P.ndm + a.dm_idx;
        else bad = true;
    }
    if (i < P.n) {
        const dedisp_event b = P.ev[i];
        if (event_ok(b, P)) {
            kcur = static_cast<int64_t>(b.width_idx) * P.ndm + b.dm_idx;
            if (i > 0) {
                const dedisp_event a = P.ev[i - 1];
                if (kcur < kprev || (kcur == kprev && b.t_start <= a.t_end)) bad = true;
            }
        } else {
            bad = true;
        }
    }
    if (bad) {
        atomicOr(err, 1u);
        return;
    }
    for (int64_t k = kprev + 1; k <= kcur; ++k) seg[k] = static_cast<int32_t>(i);
}

// Neighbour series whose events can have larger indices than an event of
// series (w, d): (w, d .. d + dm_radius) and (w + 1 .. w + width_radius,
// d - dm_radius .. d + dm_radius) -- every series of smaller key holds only
// smaller indices.
__host__ __device__ inline int upper_series(int dm_radius, int width_radius) {
    return dm_radius + 1 + width_radius * (2 * dm_radius + 1);
}

__device__ void link_one(const ClusterParams& P, const int32_t* __restrict__ seg, int32_t* parent,
                         int64_t i, int sidx);

// Thread q handles event q / S and its neighbour series q % S (S =
// upper_series): it unites the event with every friend of larger index in
// that series.  One series per thread keeps each thread's chain of dependent
// loads short.
__global__ __launch_bounds__(kKThreads) void cluster_link_kernel(ClusterParams P,
                                                                 const int32_t* __restrict__ seg,
                                                                 int32_t* parent) {
    const int S = upper_series(P.dm_radius, P.width_radius);
    const int64_t nq = P.n * S;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * kKThreads;
    for (int64_t q = static_cast<int64_t>(blockIdx.x) * kKThreads + threadIdx.x; q < nq; q += stride)
        link_one(P, seg, parent, q / S, static_cast<int>(q % S));
}

__device__ void link_one(const ClusterParams& P, const int32_t* __restrict__ seg, int32_t* parent,
                         int64_t i, int sidx) {
    const dedisp_event e = P.ev[i];
    if (!event_ok(e, P)) return;
    int w = e.width_idx, d;
    if (sidx <= P.dm_radius) {
        d = e.dm_idx + sidx;
    } else {
        const int r = sidx - P.dm_radius - 1;
        w += 1 + r / (2 * P.dm_radius + 1);
        d = e.dm_idx - P.dm_radius + r % (2 * P.dm_radius + 1);
    }
    if (w >= P.nwidths || d < 0 || d >= P.ndm) return;
    const int64_t n = P.n;
    const int64_t k = static_cast<int64_t>(w) * P.ndm + d;
    int64_t a = min<int64_t>(max<int64_t>(seg[k], 0), n);
    const int64_t b = min<int64_t>(max<int64_t>(seg[k + 1], a), n);
    if (sidx == 0) a = max(a, i + 1);            // own series: later runs only
    const int64_t want_end = e.t_start - P.time_tol - P.widths[w] + 1;   // friend: t_end >= this
    const int64_t last_start = e.t_end + P.widths[e.width_idx] - 1 + P.time_tol;
    int64_t lo = a, hi = b;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (P.ev[mid].t_end < want_end) lo = mid + 1;
        else hi = mid;
    }
    for (int64_t j = lo; j < b && P.ev[j].t_start <= last_start; ++j) {
        // most friends are already joined: a common ancestor seen through
        // ordinary cached loads settles that without the coherent union
        const int32_t ra = find_cached(parent, static_cast<int32_t>(i));
        const int32_t rb = find_cached(parent, static_cast<int32_t>(j));
        if (ra != rb) unite(parent, ra, rb);
    }
}

// Final roots, the accumulators of every root slot, and the root flags.
__global__ __launch_bounds__(kKThreads) void cluster_finish_kernel(
    int64_t n, int32_t* parent, uint32_t* __restrict__ flag, uint32_t* __restrict__ cnt,
    int32_t* __restrict__ dmlo, int32_t* __restrict__ dmhi, int32_t* __restrict__ wlo,
    int32_t* __restrict__ whi, uint64_t* __restrict__ tlo, uint64_t* __restrict__ thi,
    uint64_t* __restrict__ key) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kKThreads + threadIdx.x;
    if (i >= n) return;
    int32_t r = static_cast<int32_t>(i);
    int32_t p = atomic_ld(parent + r);
    while (p != r) {
        r = p;
        p = atomic_ld(parent + r);
    }
    atomic_st(parent + i, r);   // an ancestor of i, as every parent value is
    flag[i] = r == i;
    cnt[i] = 0;
    dmlo[i] = INT_MAX;
    dmhi[i] = INT_MIN;
    wlo[i] = INT_MAX;
    whi[i] = INT_MIN;
    tlo[i] = ~0ull;
    thi[i] = 0;
    key[i] = 0;
}

// Events per block of the accumulation and its LDS table (load <= 1/2).
constexpr int kAccEvents = 512;
constexpr int kAccSlots = 1024;

// Member count, bounds and representative of every cluster.  A block first
// merges its events per root in an LDS hash table (roots are event indices;
// linear probing), then adds each distinct root once to the global slots:
// one global atomic per field and root per block instead of per event, which
// matters when large clusters would serialise on their root's slot.
__global__ __launch_bounds__(kKThreads) void cluster_accumulate_kernel(
    ClusterParams P, const int32_t* __restrict__ parent, const int64_t* __restrict__ offs,
    uint32_t* cnt, int32_t* dmlo, int32_t* dmhi, int32_t* wlo, int32_t* whi, uint64_t* tlo,
    uint64_t* thi, uint64_t* key, int32_t* __restrict__ labels) {
    __shared__ int32_t s_root[kAccSlots];
    __shared__ uint32_t s_cnt[kAccSlots];
    __shared__ int32_t s_dmlo[kAccSlots], s_dmhi[kAccSlots], s_wlo[kAccSlots], s_whi[kAccSlots];
    __shared__ unsigned long long s_tlo[kAccSlots], s_thi[kAccSlots], s_key[kAccSlots];
    for (int h = threadIdx.x; h < kAccSlots; h += kKThreads) {
        s_root[h] = -1;
        s_cnt[h] = 0;
        s_dmlo[h] = INT_MAX;
        s_dmhi[h] = INT_MIN;
        s_wlo[h] = INT_MAX;
        s_whi[h] = INT_MIN;
        s_tlo[h] = ~0ull;
        s_thi[h] = 0;
        s_key[h] = 0;
    }
    __syncthreads();
    const int64_t i0 = static_cast<int64_t>(blockIdx.x) * kAccEvents;
    for (int k = threadIdx.x; k < kAccEvents; k += kKThreads) {
        const int64_t i = i0 + k;
        if (i >= P.n) break;
        const int32_t r = parent[i];
        if (labels) labels[i] = static_cast<int32_t>(offs[r]);
        const dedisp_event e = P.ev[i];
        if (!event_ok(e, P)) continue;
        uint32_t h = (static_cast<uint32_t>(r) * 2654435761u) >> 22;   // 10 bits
        while (true) {
            const int32_t old = atomicCAS(s_root + h, -1, r);
            if (old == -1 || old == r) break;
            h = (h + 1) & (kAccSlots - 1);
        }
        atomicAdd(s_cnt + h, 1u);
        atomicMin(s_dmlo + h, e.dm_idx);
        atomicMax(s_dmhi + h, e.dm_idx);
        atomicMin(s_wlo + h, e.width_idx);
        atomicMax(s_whi + h, e.width_idx);
        atomicMin(s_tlo + h, static_cast<unsigned long long>(e.t_start));
        atomicMax(s_thi + h, static_cast<unsigned long long>(e.t_end + P.widths[e.width_idx] - 1));
        atomicMax(s_key + h, static_cast<unsigned long long>(rep_key(e.snr, i)));
    }
    __syncthreads();
    for (int h = threadIdx.x; h < kAccSlots; h += kKThreads) {
        const int32_t r = s_root[h];
        if (r < 0 || s_cnt[h] == 0) continue;
        atomicAdd(cnt + r, s_cnt[h]);
        atomicMin(dmlo + r, s_dmlo[h]);
        atomicMax(dmhi + r, s_dmhi[h]);
        atomicMin(wlo + r, s_wlo[h]);
        atomicMax(whi + r, s_whi[h]);
        atomicMin(reinterpret_cast<unsigned long long*>(tlo + r), s_tlo[h]);
        atomicMax(reinterpret_cast<unsigned long long*>(thi + r), s_thi[h]);
        atomicMax(reinterpret_cast<unsigned long long*>(key + r), s_key[h]);
    }
}

__global__ __launch_bounds__(kKThreads) void cluster_write_kernel(
    ClusterParams P, const uint32_t* __restrict__ flag, const int64_t* __restrict__ offs,
    const uint32_t* __restrict__ cnt, const int32_t* __restrict__ dmlo,
    const int32_t* __restrict__ dmhi, const int32_t* __restrict__ wlo,
    const int32_t* __restrict__ whi, const uint64_t* __restrict__ tlo,
    const uint64_t* __restrict__ thi, const uint64_t* __restrict__ key,
    dedisp_cluster* __restrict__ out, int64_t capacity) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kKThreads + threadIdx.x;
    if (i >= P.n || !flag[i]) return;
    const int64_t c = offs[i];
    if (c >= capacity) return;
    // key 0 only when no valid member reached the slot (rejected input): stay in bounds
    const int64_t rep = key[i] ? 0xFFFFFFFFll - static_cast<int64_t>(key[i] & 0xFFFFFFFFull) : i;
    const dedisp_event e = P.ev[rep];
    dedisp_cluster o;
    o.first = i;
    o.rep = rep;
    o.t_lo = static_cast<int64_t>(tlo[i]);
    o.t_hi = static_cast<int64_t>(thi[i]);
    o.t_peak = e.t_peak;
    o.n_members = static_cast<int32_t>(cnt[i]);
    o.dm_lo = dmlo[i];
    o.dm_hi = dmhi[i];
    o.w_lo = wlo[i];
    o.w_hi = whi[i];
    o.dm_idx = e.dm_idx;
    o.width_idx = e.width_idx;
    o.snr = e.snr;
    out[c] = o;
}

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

struct ClusterLayout {
    size_t o_seg, o_parent, o_flag, o_cnt, o_dmlo, o_dmhi, o_wlo, o_whi, o_tlo, o_thi, o_key,
        o_offs, o_chunk, o_total, o_err, bytes;
};

ClusterLayout cluster_layout(int64_t n, int32_t ndm, int32_t nwidths) {
    ClusterLayout L{};
    const size_t un = static_cast<size_t>(std::max<int64_t>(n, 1));
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o = align256(o + bytes);
        return at;
    };
    L.o_seg = take((static_cast<size_t>(ndm) * nwidths + 1) * 4);
    L.o_parent = take(un * 4);
    L.o_flag = take(un * 4);
    L.o_cnt = take(un * 4);
    L.o_dmlo = take(un * 4);
    L.o_dmhi = take(un * 4);
    L.o_wlo = take(un * 4);
    L.o_whi = take(un * 4);
    L.o_tlo = take(un * 8);
    L.o_thi = take(un * 8);
    L.o_key = take(un * 8);
    L.o_offs = take(un * 8);
    L.o_chunk = take(static_cast<size_t>(dd::scan_chunk_count(static_cast<int64_t>(un))) * 8);
    L.o_total = take(16);   // int64 count, then the uint32 error flag
    L.o_err = L.o_total + 8;
    L.bytes = o;
    return L;
}

}  // namespace

namespace dd {

size_t cluster_workspace_bytes(int64_t n, int32_t ndm, int32_t nwidths) {
    return cluster_layout(n, ndm, nwidths).bytes;
}

// Launch the whole stage.  *result (device) receives, when the stream reaches
// it, two int64: the cluster count, then the input-error flag (low 32 bits).
hipError_t launch_cluster(const dedisp_event* ev, int64_t n, int32_t ndm, const int32_t* widths,
                          int32_t nwidths, int32_t dm_radius, int32_t width_radius, int64_t time_tol,
                          dedisp_cluster* out, int64_t capacity, int32_t* labels, void* ws,
                          const int64_t** result, hipStream_t s) {
    const ClusterLayout L = cluster_layout(n, ndm, nwidths);
    char* b = static_cast<char*>(ws);
    auto at = [&](size_t o) { return static_cast<void*>(b + o); };
    int32_t* seg = static_cast<int32_t*>(at(L.o_seg));
    int32_t* parent = static_cast<int32_t*>(at(L.o_parent));
    uint32_t* flag = static_cast<uint32_t*>(at(L.o_flag));
    uint32_t* cnt = static_cast<uint32_t*>(at(L.o_cnt));
    int32_t* dmlo = static_cast<int32_t*>(at(L.o_dmlo));
    int32_t* dmhi = static_cast<int32_t*>(at(L.o_dmhi));
    int32_t* wlo = static_cast<int32_t*>(at(L.o_wlo));
    int32_t* whi = static_cast<int32_t*>(at(L.o_whi));
    uint64_t* tlo = static_cast<uint64_t*>(at(L.o_tlo));
    uint64_t* thi = static_cast<uint64_t*>(at(L.o_thi));
    uint64_t* key = static_cast<uint64_t*>(at(L.o_key));
    int64_t* offs = static_cast<int64_t*>(at(L.o_offs));
    int64_t* chunk = static_cast<int64_t*>(at(L.o_chunk));
    int64_t* total = static_cast<int64_t*>(at(L.o_total));
    uint32_t* err = static_cast<uint32_t*>(at(L.o_err));
    *result = total;

    ClusterParams P{};
    P.ev = ev;
    P.n = n;
    P.ndm = ndm;
    P.nwidths = nwidths;
    P.dm_radius = dm_radius;
    P.width_radius = width_radius;
    P.time_tol = time_tol;
    for (int k = 0; k < nwidths; ++k) P.widths[k] = widths[k];

    const dim3 blk(kKThreads);
    const dim3 g_n(static_cast<unsigned>((n + kKThreads - 1) / kKThreads));
    const dim3 g_n1(static_cast<unsigned>((n + 1 + kKThreads - 1) / kKThreads));
    hipLaunchKernelGGL(cluster_init_kernel, dim3(1), dim3(1), 0, s, err);
    hipLaunchKernelGGL(cluster_seg_kernel, g_n1, blk, 0, s, P, seg, parent, err);
    const int64_t nq = n * upper_series(dm_radius, width_radius);
    const int64_t link_blocks = std::min<int64_t>((nq + kKThreads - 1) / kKThreads, int64_t(1) << 20);
    hipLaunchKernelGGL(cluster_link_kernel, dim3(static_cast<unsigned>(link_blocks)), blk, 0, s, P,
                       seg, parent);
    hipLaunchKernelGGL(cluster_finish_kernel, g_n, blk, 0, s, n, parent, flag, cnt, dmlo, dmhi,
                       wlo, whi, tlo, thi, key);
    hipError_t e = launch_scan_u32(flag, n, offs, chunk, total, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(cluster_accumulate_kernel,
                       dim3(static_cast<unsigned>((n + kAccEvents - 1) / kAccEvents)), blk, 0, s,
                       P, parent, offs, cnt, dmlo, dmhi,
                       wlo, whi, tlo, thi, key, labels);
    if (capacity > 0)
        hipLaunchKernelGGL(cluster_write_kernel, g_n, blk, 0, s, P, flag, offs, cnt, dmlo, dmhi, wlo,
                           whi, tlo, thi, key, out, capacity);
    return hipGetLastError();
}

}  // namespace dd

extern "C" size_t dedisp_cluster_workspace_bytes(int64_t n_events, int32_t ndm, int32_t nwidths) {
    if (n_events < 0 || n_events > INT32_MAX || ndm < 1 || ndm > 65535 || nwidths < 1 ||
        nwidths > dd::kMaxWidths)
        return 0;
    return dd::cluster_workspace_bytes(n_events, ndm, nwidths);
}

extern "C" dedisp_status dedisp_cluster_events(const dedisp_event* events, int64_t n_events,
                                               int32_t ndm, const int32_t* widths, int32_t nwidths,
                                               int32_t dm_radius, int32_t width_radius,
                                               int64_t time_tol, dedisp_cluster* clusters,
                                               int64_t capacity, int64_t* n_clusters,
                                               int32_t* labels, void* workspace,
                                               dedisp_stream stream) {
    using dd::fail;
    if (!n_clusters || !widths) return fail(DEDISP_ERR_INVALID_ARG, "NULL argument");
    if (n_events < 0 || n_events > INT32_MAX)
        return fail(DEDISP_ERR_INVALID_ARG, "n_events %lld outside [0, 2^31 - 1]",
                    static_cast<long long>(n_events));
    if (capacity < 0) return fail(DEDISP_ERR_INVALID_ARG, "capacity < 0");
    if (ndm < 1 || ndm > 65535 || nwidths < 1 || nwidths > dd::kMaxWidths)
        return fail(DEDISP_ERR_INVALID_ARG, "need 1 <= ndm <= 65535 and 1 <= nwidths <= 32");
    for (int k = 0; k < nwidths; ++k)
        if (widths[k] < 1 || widths[k] > (1 << 30))
            return fail(DEDISP_ERR_INVALID_ARG, "width %d outside [1, 2^30]", widths[k]);
    if (dm_radius < 0 || dm_radius > 65535 || width_radius < 0 || width_radius > 31 ||
        time_tol < 0 || time_tol > (int64_t(1) << 40))
        return fail(DEDISP_ERR_INVALID_ARG, "radius or tolerance out of range");
    *n_clusters = 0;
    if (n_events == 0) {
        dd::clear_error();
        return DEDISP_OK;
    }
    if (!events || !workspace || (capacity > 0 && !clusters))
        return fail(DEDISP_ERR_INVALID_ARG, "NULL argument");
    if (reinterpret_cast<uintptr_t>(workspace) % 256)
        return fail(DEDISP_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
    const int64_t* d_result = nullptr;
    DD_HIP(dd::launch_cluster(events, n_events, ndm, widths, nwidths, dm_radius, width_radius,
                              time_tol, clusters, capacity, labels, workspace, &d_result, stream));
    int64_t back[2] = {0, 0};   // count, error flag
    DD_HIP(hipMemcpyAsync(back, d_result, sizeof back, hipMemcpyDeviceToHost, stream));
    DD_HIP(hipStreamSynchronize(stream));
    const int64_t total = back[0];
    const uint32_t err = static_cast<uint32_t>(back[1]);
    if (err)
        return fail(DEDISP_ERR_INVALID_ARG,
                    "events are not in find_peaks order or have fields out of range");
    *n_clusters = total;
    if (total > capacity)
        return fail(DEDISP_ERR_CAPACITY, "%lld clusters found, capacity %lld",
                    static_cast<long long>(total), static_cast<long long>(capacity));
    dd::clear_error();
    return DEDISP_OK;
}

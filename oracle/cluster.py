"""Event clustering across DM and width (oracle; test infrastructure).

Section 2.3 ends the search by gathering contiguous above-threshold samples
of one series into events.  A real dispersed pulse crosses the cut in many
neighbouring DM trials and boxcar widths at once, so one pulse yields many
events; this step merges them into one candidate.  The paper only names the
per-series gathering; the merging rule is a stated reading:

  * event e covers the samples [t_start, t_end + W - 1] of the dedispersed
    series, W = widths[width_idx] (the boxcar starting at t sums samples
    t .. t + W - 1);
  * events a and b are friends when |dm_a - dm_b| <= dm_radius,
    |width_idx_a - width_idx_b| <= width_radius and their sample spans are no
    more than time_tol samples apart: s_a <= e_b + time_tol and
    s_b <= e_a + time_tol;
  * a cluster is a connected component of the friend relation (friends of
    friends belong together);
  * clusters are listed in the order of their lowest-index member; the
    representative is the member of largest snr, ties to the lower index.

The definition is a plain one (connected components of a graph), so the
oracle writes it out: every pair is tested, the components come from a
library connected-components routine, and the records are filled by plain
loops.  Input events are in the find_peaks order and layout (EVENT_FIELDS).
"""
from __future__ import annotations

import numpy as np
from scipy.sparse import coo_matrix
from scipy.sparse.csgraph import connected_components

CLUSTER_FIELDS = ("first", "rep", "n_members", "dm_lo", "dm_hi", "w_lo", "w_hi", "t_lo",
                  "t_hi", "t_peak", "dm_idx", "width_idx", "snr")


def spans(events, widths):
    """(start, end inclusive) sample span of every event, int64 arrays."""
    ev = _columns(events)
    w = np.asarray(widths, np.int64)[ev["width_idx"]]
    return ev["t_start"], ev["t_end"] + w - 1


def friend_pairs(events, widths, dm_radius: int, width_radius: int, time_tol: int):
    """All friend pairs (i, j), i < j, by testing every pair."""
    ev = _columns(events)
    n = len(ev["dm_idx"])
    s, e = spans(events, widths)
    ii, jj = [], []
    block = 512
    for a in range(0, n, block):
        b = min(n, a + block)
        d = np.abs(ev["dm_idx"][a:b, None] - ev["dm_idx"][None, :]) <= dm_radius
        w = np.abs(ev["width_idx"][a:b, None] - ev["width_idx"][None, :]) <= width_radius
        t = (s[a:b, None] <= e[None, :] + time_tol) & (s[None, :] <= e[a:b, None] + time_tol)
        upper = np.arange(a, b)[:, None] < np.arange(n)[None, :]
        r, c = np.nonzero(d & w & t & upper)
        ii.append(r + a)
        jj.append(c)
    if not ii:
        return np.zeros(0, np.int64), np.zeros(0, np.int64)
    return np.concatenate(ii).astype(np.int64), np.concatenate(jj).astype(np.int64)


def cluster_events(events, widths, dm_radius: int, width_radius: int, time_tol: int):
    """Returns (labels [n] int64 = cluster index of each event, clusters: a
    list of dicts keyed by CLUSTER_FIELDS, in cluster-index order)."""
    ev = _columns(events)
    n = len(ev["dm_idx"])
    if n == 0:
        return np.zeros(0, np.int64), []
    i, j = friend_pairs(events, widths, dm_radius, width_radius, time_tol)
    g = coo_matrix((np.ones(len(i), np.int8), (i, j)), shape=(n, n))
    _, comp = connected_components(g, directed=False)
    # number the components by their lowest member
    first = {}
    for k in range(n):
        first.setdefault(int(comp[k]), k)
    order = sorted(first.values())
    index = {int(comp[f]): c for c, f in enumerate(order)}
    labels = np.array([index[int(comp[k])] for k in range(n)], np.int64)
    s, e = spans(events, widths)
    groups = [[] for _ in order]
    for k in range(n):
        groups[labels[k]].append(k)
    clusters = []
    for c, f in enumerate(order):
        members = np.array(groups[c], np.int64)
        rep = int(members[0])
        for m in members[1:]:
            if ev["snr"][m] > ev["snr"][rep]:
                rep = int(m)
        clusters.append(dict(
            first=int(f), rep=rep, n_members=len(members),
            dm_lo=int(ev["dm_idx"][members].min()), dm_hi=int(ev["dm_idx"][members].max()),
            w_lo=int(ev["width_idx"][members].min()), w_hi=int(ev["width_idx"][members].max()),
            t_lo=int(s[members].min()), t_hi=int(e[members].max()),
            t_peak=int(ev["t_peak"][rep]), dm_idx=int(ev["dm_idx"][rep]),
            width_idx=int(ev["width_idx"][rep]), snr=float(ev["snr"][rep])))
    return labels, clusters


def _columns(events):
    """Event columns as arrays, from a structured array or a list of tuples."""
    names = ("width_idx", "dm_idx", "t_start", "t_end", "t_peak", "b_peak", "snr")
    if isinstance(events, np.ndarray) and events.dtype.names:
        return {k: np.asarray(events[k], np.float32 if k == "snr" else np.int64) for k in names}
    rows = list(events)
    out = {}
    for c, k in enumerate(names):
        out[k] = np.array([r[c] for r in rows], np.float32 if k == "snr" else np.int64)
    return out

"""Device-memory helpers around the C ABI.

`Search` keeps a plan plus reusable device buffers (torch tensors) and runs
the chain dedisperse -> find_peaks on one beam.  It only allocates memory and
calls the library; every step of the computation runs in the HIP kernels.
"""
from __future__ import annotations

from typing import Optional, Sequence

import numpy as np

from . import _lib as L


class Search:
    def __init__(self, nchans: int, f_top: float, df: float, tsamp: float, dm_list,
                 widths: Sequence[int], snr_thresh: float, out_u16: bool = True,
                 device: str = "cuda", capacity: int = 1 << 20):
        import torch
        self.torch = torch
        self.plan = L.dedisp_plan_create(nchans, f_top, df, tsamp, dm_list)
        self.nchans = nchans
        self.ndm = self.plan.ndm
        self.max_delay = self.plan.max_delay
        self.widths = [int(w) for w in widths]
        self.snr_thresh = float(snr_thresh)
        self.out_dtype = torch.uint16 if out_u16 else torch.int32
        self.device = device
        self.capacity = int(capacity)
        self._ws = None
        self._pk_ws = None
        self._events = None

    def _buf(self, attr: str, nbytes: int):
        t = getattr(self, attr)
        if t is None or t.numel() < nbytes:
            t = self.torch.empty(max(nbytes, 256), dtype=self.torch.uint8, device=self.device)
            setattr(self, attr, t)
        return t

    def nout(self, nsamps: int) -> int:
        return int(nsamps) - self.max_delay

    def dedisperse(self, packed, nsamps: int, out=None, tile=None, stream=None):
        nout = self.nout(nsamps)
        if out is None:
            out = self.torch.empty((self.ndm, nout), dtype=self.out_dtype, device=self.device)
        ws = self._buf("_ws", L.dedisp_workspace_bytes(self.plan, nsamps))
        if tile is None:
            L.dedisp_execute(self.plan, packed, nsamps, out, ws, stream)
        else:
            L.dedisp_execute_tile(self.plan, packed, nsamps, out, ws, tile, stream)
        return out

    def find_peaks(self, series, capacity: Optional[int] = None, stream=None):
        nout = series.shape[1]
        cap = self.capacity if capacity is None else int(capacity)
        ws = self._buf("_pk_ws", L.find_peaks_workspace_bytes(self.ndm, nout, self.widths))
        ev = self._buf("_events", max(cap, 1) * L.EVENT_DTYPE.itemsize)
        n = L.find_peaks(series, self.ndm, nout, self.widths, self.snr_thresh, ev, cap, ws,
                         stream)
        return L.events_from_buffer(ev, n)

    def stats(self, nout: int):
        return L.find_peaks_read_stats(self._pk_ws, self.ndm, nout, self.widths)

    def run(self, packed, nsamps: int, stream=None):
        out = self.dedisperse(packed, nsamps, stream=stream)
        return out, self.find_peaks(out, stream=stream)

"""Torch-side holder of one domain: device particle arrays plus a library context.

Plumbing only -- it allocates torch device tensors, fills an ``sph_particles``
record and forwards to the C ABI; every step of the update runs in the HIP
library.
"""
from __future__ import annotations

from typing import List, Optional, Sequence

import numpy as np
import torch

from . import sphbuf as S


class Domain:
    def __init__(self, dim: int, lo, hi, cell_size: float, dp: float, capacity: int,
                 pos: Sequence[np.ndarray], carried: Sequence[np.ndarray], label: np.ndarray, ids: np.ndarray,
                 n: int, next_id: int, max_events: int = 4096, device: str = "cuda:0",
                 stream: Optional[torch.cuda.Stream] = None, brick_log2: int = 0, brick_margin: int = 1,
                 update_path: str = "merged", build_method: str = "auto"):
        self.dim = dim
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        dev = self.device
        self.pos = [torch.zeros(capacity, dtype=torch.float32, device=dev) for _ in range(dim)]
        self.carried = [torch.zeros(capacity, dtype=torch.float32, device=dev) for _ in carried]
        self.label = torch.zeros(capacity, dtype=torch.int32, device=dev)
        self.id = torch.full((capacity,), -1, dtype=torch.int64, device=dev)
        self.n_dev = torch.zeros(1, dtype=torch.int64, device=dev)
        self.capacity = capacity
        self.upload(pos, carried, label, ids, n)
        st, ctx = S.sph_create(dim, lo, hi, cell_size, dp, capacity, max_events, next_id,
                               self.stream.cuda_stream, brick_log2, brick_margin, S.UPDATE_PATHS[update_path],
                               S.BUILD_METHODS[build_method])
        S.check(st, "sph_create")
        self.ctx = ctx
        self.p = S.particles_from_tensors(self.pos, self.carried, self.label, self.id, self.n_dev)
        self.buffer_ids: List[int] = []

    # -- data movement (harness) --------------------------------------------
    def upload(self, pos, carried, label, ids, n: int) -> None:
        with torch.cuda.stream(self.stream):
            for t, a in zip(self.pos, pos):
                t.copy_(torch.from_numpy(np.ascontiguousarray(a[: self.capacity])))
            for t, a in zip(self.carried, carried):
                t.copy_(torch.from_numpy(np.ascontiguousarray(a[: self.capacity])))
            self.label.copy_(torch.from_numpy(np.ascontiguousarray(label[: self.capacity])))
            self.id.copy_(torch.from_numpy(np.ascontiguousarray(ids[: self.capacity])))
            self.n_dev.fill_(int(n))
        self.stream.synchronize()

    def n(self) -> int:
        self.stream.synchronize()
        return int(self.n_dev.item())

    def download(self):
        """Host copies: (pos list, carried list, label, id, n) of the whole capacity."""
        self.stream.synchronize()
        pos = [t.cpu().numpy() for t in self.pos]
        car = [t.cpu().numpy() for t in self.carried]
        return pos, car, self.label.cpu().numpy(), self.id.cpu().numpy(), int(self.n_dev.item())

    # -- C ABI --------------------------------------------------------------
    def define(self, kind: int, origin, rot, half, margin: float) -> int:
        st, bid = S.sph_buffer_define(self.ctx, kind, origin, rot, half, margin)
        S.check(st, "sph_buffer_define")
        self.buffer_ids.append(bid)
        return bid

    def fit(self) -> None:
        S.check(S.sph_grid_fit(self.ctx, self.p), "sph_grid_fit")

    def build(self) -> None:
        S.check(S.sph_celllist_build(self.ctx, self.p), "sph_celllist_build")

    def identify(self, buffer_id: int = -1) -> int:
        return S.sph_buffer_identify(self.ctx, self.p, buffer_id)

    def update(self):
        return S.sph_buffer_update(self.ctx, self.p)

    def update_async(self) -> int:
        return S.sph_buffer_update_async(self.ctx, self.p)

    def update_fullscan(self):
        return S.sph_buffer_update_fullscan(self.ctx, self.p)

    def update_fullscan_async(self) -> int:
        return S.sph_buffer_update_fullscan_async(self.ctx, self.p)

    def set_fields(self, vel, rho: int = -1) -> None:
        S.check(S.sph_set_fields(self.ctx, vel, rho), "sph_set_fields")

    def set_bc(self, buffer_id: int, kind: int, **kw) -> None:
        S.check(S.sph_buffer_set_bc(self.ctx, buffer_id, kind, **kw), "sph_buffer_set_bc")

    def apply_bc(self) -> int:
        return S.sph_buffer_apply_bc(self.ctx, self.p)

    def rotate(self, buffer_id: int, center, m) -> int:
        return S.sph_buffer_rotate(self.ctx, self.p, buffer_id, center, m)

    def rotate_async(self, buffer_id: int, center, m) -> int:
        return S.sph_buffer_rotate_async(self.ctx, self.p, buffer_id, center, m)

    def apply_bc_async(self) -> int:
        return S.sph_buffer_apply_bc_async(self.ctx, self.p)

    def bc_status(self) -> int:
        return S.sph_last_bc_status(self.ctx)

    def neighbor_count(self, radius: float):
        """(status, int32 device tensor of the capacity; entries below N hold the counts)."""
        counts = torch.full((self.capacity,), -1, dtype=torch.int32, device=self.device)
        st = S.sph_neighbor_count(self.ctx, self.p, radius, counts.data_ptr())
        self.stream.synchronize()
        return st, counts

    def result(self):
        return S.sph_last_result(self.ctx)

    def events(self, cap: int = S.SPH_MAX_EVENTS_LIMIT):
        return S.sph_last_events(self.ctx, cap)

    def close(self) -> None:
        if getattr(self, "ctx", None):
            S.sph_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

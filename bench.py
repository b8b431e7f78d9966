#!/usr/bin/env python
"""Benchmark of the buffer-update hot path on one MI355X.

One step = one pass of the whole path over one particle state: the cell-list
build (count, scan, scatter) followed by the buffer update (local-cell
candidates, frame rotation, crossing tests, generation/recycle, deletion by
compaction, relabel), on the library's default path (the merged step).

Headline workload: the 3-D bifurcating pipe network (trunk, two daughters, two
granddaughters; dp = 0.001, about 16.1 M particles on a brick-sparse grid; one
bidirectional buffer at the trunk inlet and one at each of the three leaf
outlets; reversing sinusoidal flow of period 200 steps).  The 3-D pipe (7.86 M
particles, inlet and outlet tilted 20 and 35 degrees) is a second leg with the
same measurements.

The particle states the timed steps consume are prepared beforehand by running
the real loop (update, then advection with the prescribed velocity) from the
initial lattice and keeping a device copy of each pre-update state.  The timed
window starts late in the run (step 445 of the network, at peak flow after two
reversals; step 400 of the pipe), when the particles have left their initial
lattice order; an early window (from step 5) is timed as well and reported as
the drift.  The timed region replays the window's states in order, so every
timed step does the full work of a real step (events included) on inputs
already resident in HBM, and nothing else.

Printed: one JSON line with the throughput, the roofline of the dominant
kernel, the full-scan baseline, the legs, and the FP64 CPU oracle timed on this
host (one thread and all threads; brute force and the local-cell method).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "buffer-update Mparticles/s, speedup vs full scan, % HBM peak; batched vs plain"

DESCRIPTION = {
    "tree3d": "3-D bifurcating pipe network (trunk R=0.05, daughters R=0.04, granddaughters R=0.03), dp=0.001, "
              "4 bidirectional buffers (trunk inlet, 3 leaf outlets), reversing flow of period 200 steps, "
              "brick-sparse grid",
    "pipe3d": "3-D pipe R=0.05 L=1.0 dp=0.001, inlet tilted 20 deg about x, outlet 35 deg about y",
    "bent_channel2d": "2-D bent channel W=0.2, dp=0.002, inlet at 30 deg, outlet at -45 deg",
    "channel2d": "2-D straight channel 2.0 x 0.4, dp=0.02, axis-aligned inlet and outlet",
}
LATE_START = {"tree3d": 445, "pipe3d": 400, "bent_channel2d": 400, "channel2d": 100}
BRICKS = {"tree3d": 3}


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


class ProfilerRegions:
    """roctx pause/resume requests around the timed loops, so that a profiler run
    with --selected-regions sees exactly the timed launches (and one calibration
    copy of known size).  Without a profiler attached the requests do nothing."""

    def __init__(self):
        import ctypes
        self.lib = None
        for name in ("librocprofiler-sdk-roctx.so.1", "librocprofiler-sdk-roctx.so"):
            try:
                self.lib = ctypes.CDLL(name)
                break
            except OSError:
                continue
        if self.lib is not None:
            self.lib.roctxProfilerPause.argtypes = [ctypes.c_uint64]
            self.lib.roctxProfilerResume.argtypes = [ctypes.c_uint64]

    def begin(self):
        if self.lib is not None:
            self.lib.roctxProfilerResume(0)

    def end(self):
        if self.lib is not None:
            self.lib.roctxProfilerPause(0)


REGIONS = ProfilerRegions()


def rotation_of(S, spec, dim):
    if dim == 2:
        st, q = S.sph_rotation_2d(spec.angle)
    else:
        st, q = S.sph_rotation_from_direction(spec.direction)
    S.check(st, "rotation")
    return q


def make_workload(name: str):
    import workloads as W
    return {"tree3d": W.tree3d, "pipe3d": W.pipe3d, "bent_channel2d": W.bent_channel2d,
            "channel2d": W.channel2d}[name]()


class Snapshot:
    """Device copy of one particle state."""

    def __init__(self, dom):
        self.pos = [t.clone() for t in dom.pos]
        self.carried = [t.clone() for t in dom.carried]
        self.label = dom.label.clone()
        self.id = dom.id.clone()
        self.n_dev = dom.n_dev.clone()

    def tensors(self):
        return self.pos + self.carried + [self.label, self.id, self.n_dev]


def phase_bytes(dim: int, n: int, n_cells: int, cand: int, g: int, d: int, n_carried: int,
                method: str = "bucketed"):
    """Algorithmic bytes per launch of each kernel phase: its inputs and outputs in
    HBM, the build's intermediates included ("build" is the least any build must
    move: positions in, cell list out).  The build's phases differ by method."""
    state = 4 * dim + 4 * n_carried + 4 + 8          # bytes of one particle's state
    if method == "counting":
        build = {
            "count": (4 * dim + 4) * n + 4 * n_cells,   # read positions, write packed (key, rank); the counters
            "scan": 8 * (n_cells + 1),                  # read counts, write cell starts
            "scatter": 8 * n + 4 * (n_cells + 1),       # read packed words and cell starts, write cell_idx
        }
    else:
        build = {
            "count": (4 * dim + 8) * n,                 # read positions, write (key, rank in bucket)
            "scatter": 16 * n,                          # read (key, rank), write (key, particle) in bucket order
            "sort": 12 * n + 4 * (n_cells + 1),         # read (key, particle), write cell_idx and cell_start
        }
    return {
        "build": (4 * dim + 4) * n + 4 * (n_cells + 1), # read positions, write cell_idx and cell_start
        "scan": 8 * (n_cells + 1),                      # (batched build) read counts, write cell starts
        **build,
        "classify": cand * (4 * dim + 8),               # candidate index, position, label
        "candidates": cand * (4 * dim + 8),
        "fullscan": 4 * dim * n,                        # read positions
        "finalize": (g + d) * 8 + g * (2 * state) + d * 2 * state,  # events, duplicates, refills
    }


TUNE_BUILDS = 10
# the merged step's kernels per phase, by build method
KERNEL_OF = {
    "bucketed": {"count": "k_bk_count<true>", "scatter": "k_bk_scatter_cls", "sort": "k_bk_sort",
                 "finalize": "k_finalize"},
    "counting": {"count": "k_count<true>", "scan": "k_scan", "scatter": "k_scatter_cls", "finalize": "k_finalize"},
}
PHASES_NOTE = {
    "bucketed": "merged step, bucketed build: count = bucket counts and the candidate list, scatter = the bucket "
                "scatter with the candidates' exact tests beside it, sort = the per-bucket counting sort, "
                "finalize = the events applied",
    "counting": "merged step, counting build: count = cell counts and the candidate list, scan = the look-back "
                "scan of the counts, scatter = the cell-list scatter with the candidates' exact tests beside it, "
                "finalize = the events applied",
}


def build_method(ctx):
    """The automatic build method's choice for a context and the times it rests on."""
    from paper_2406_16786_amd import sphbuf as S
    st, m, us, ns = S.sph_build_stats(ctx)
    S.check(st, "build_stats")
    name = {S.SPH_BUILD_COUNTING: "counting", S.SPH_BUILD_BUCKETED: "bucketed"}.get(m, "none")
    return {"chosen": name, "us_counting": round(us[0], 1), "us_bucketed": round(us[1], 1),
            "timed_builds": {"counting": int(ns[0]), "bucketed": int(ns[1])}}


def measured_traffic(workload: str, kernel: str):
    """HBM bytes per launch of a kernel from the committed rocprofv3 counter
    summary, if it was taken on the current kernel source (else None)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.json")
    src_path = os.path.join(ROOT, "paper_2406_16786_amd", "csrc", "sphbuf.hip")
    try:
        t = json.load(open(path))
        if t.get("source_sha256") != hashlib.sha256(open(src_path, "rb").read()).hexdigest():
            return None
        e = max(t["workloads"][workload]["kernels"][kernel], key=lambda r: r["grid"])
        return int(e["fetch_bytes"] + e["write_bytes"])
    except (OSError, KeyError, ValueError, TypeError):
        return None


def cover_candidates(np, S, wl, rots, pos, n):
    """Particles of the buffers' cover cells (what the local path examines), from
    the dense cover of each check region and the FP32 cell of every particle."""
    dims = [int(math.ceil((wl.hi[c] - wl.lo[c]) / wl.cell_size)) for c in range(wl.dim)] + [1] * (3 - wl.dim)
    lo32 = np.asarray(wl.lo[: wl.dim], dtype=np.float32)
    ic = np.float32(1.0 / wl.cell_size)
    key = np.zeros(n, dtype=np.int64)
    mul = 1
    for c in range(wl.dim):
        t = ((pos[c][:n] - lo32[c]).astype(np.float32) * ic).astype(np.float32)
        key += np.clip(np.floor(t), 0, dims[c] - 1).astype(np.int64) * mul
        mul *= dims[c]
    total = 0
    for b, q in zip(wl.buffers, rots):
        st, f, ln = S.sph_grid_cover(wl.dim, wl.lo, wl.cell_size, dims, b.origin, q, b.half, b.margin)
        S.check(st, "grid_cover")
        cells = np.concatenate([np.arange(a, a + l) for a, l in zip(f, ln)]) if len(f) else np.zeros(0, np.int64)
        total += int(np.isin(key, cells).sum())
    return total


def single_leg(torch, np, S, W, Domain, wl, K, Wm, late, early, args):
    """Prepare the run of one workload, then time its early and late windows
    through the merged step (timed path), the cover-cell walk and the full scan."""
    dev = torch.device("cuda:0")
    t_leg = time.perf_counter()
    rots = [rotation_of(S, b, wl.dim) for b in wl.buffers]
    blog2 = BRICKS.get(wl.name, 0)
    dom = Domain(wl.dim, wl.lo, wl.hi, wl.cell_size, wl.dp, wl.capacity, wl.pos, wl.carried, wl.label, wl.id,
                 wl.n, wl.n, max_events=S.SPH_MAX_EVENTS_LIMIT, brick_log2=blog2, update_path="merged")
    for b, q in zip(wl.buffers, rots):
        dom.define(b.kind, b.origin, q, b.half, b.margin)
    st_c, ctx_cells = S.sph_create(wl.dim, wl.lo, wl.hi, wl.cell_size, wl.dp, wl.capacity,
                                   max_events=S.SPH_MAX_EVENTS_LIMIT, next_id=wl.n, stream=dom.stream.cuda_stream,
                                   brick_log2=blog2, update_path=S.SPH_UPDATE_CELLS)
    S.check(st_c, "create (cover-cell walk)")
    for b, q in zip(wl.buffers, rots):
        S.check(S.sph_buffer_define(ctx_cells, b.kind, b.origin, q, b.half, b.margin)[0], "define (cells)")
    # merged-step contexts with a fixed build method: the automatic choice's evidence
    fixed = {}
    for mname in ("counting", "bucketed"):
        st_m, ctx_m = S.sph_create(wl.dim, wl.lo, wl.hi, wl.cell_size, wl.dp, wl.capacity,
                                   max_events=S.SPH_MAX_EVENTS_LIMIT, next_id=wl.n, stream=dom.stream.cuda_stream,
                                   brick_log2=blog2, update_path=S.SPH_UPDATE_MERGED,
                                   build_method=S.BUILD_METHODS[mname])
        S.check(st_m, f"create ({mname})")
        for b, q in zip(wl.buffers, rots):
            S.check(S.sph_buffer_define(ctx_m, b.kind, b.origin, q, b.half, b.margin)[0], f"define ({mname})")
        fixed[mname] = ctx_m
    if blog2:  # every context fits its bricks to the same initial state
        dom.fit()
        S.check(S.sph_grid_fit(ctx_cells, dom.p), "grid_fit (cells)")
        for mname, ctx_m in fixed.items():
            S.check(S.sph_grid_fit(ctx_m, dom.p), f"grid_fit ({mname})")
    S.check(dom.identify(-1), "identify")
    stream = dom.stream

    # ---- the real loop, untimed: keep the states of both windows ----
    windows = {"late": late} if args.late_only else {"early": early, "late": late}
    snaps = {k: [] for k in windows}
    states = {k: [] for k in windows}
    nlist = {k: [] for k in windows}
    last = max(windows.values()) + Wm + K
    gen = torch.Generator(device=dev)
    for s in range(last):
        keep = [k for k, s0 in windows.items() if s0 <= s < s0 + Wm + K]
        for k in keep:
            st, nid, nl = S.sph_state_get(dom.ctx)
            states[k].append((nid, nl.copy()))
            snaps[k].append(Snapshot(dom))
        # the full-scan update: the same results, and the build kernels run in the
        # replays only (a kernel trace of the run then times just those)
        S.check(S.sph_buffer_update_fullscan_async(dom.ctx, dom.p), "update")
        rs, r = dom.result()
        S.check(r.status, f"update in preparation step {s}")
        for k in keep:
            nlist[k].append((r.n_before, r.n_after, r.n_generated, r.n_deleted))
        n = r.n_after
        gen.manual_seed(wl.seed_noise + s)
        with torch.cuda.stream(stream):
            p = [t[:n] for t in dom.pos]
            noise = torch.randn((wl.dim, n), generator=gen, device=dev, dtype=torch.float32)
            u = wl.velocity(torch, p, s, noise)
            for c in range(wl.dim):
                p[c].add_(u[c] * wl.dt)
    stream.synchronize()
    log(f"{wl.name}: prepared {last} steps in {time.perf_counter() - t_leg:.1f} s")

    flush = torch.ones(1 << 28, dtype=torch.float32, device=dev)       # 1 GB, read-only flush
    n_cells = int(S.sph_celllist_view(dom.ctx)[3])

    def run_window(k):
        work = [Snapshot(dom) for _ in range(Wm + K)]
        parts = [S.particles_from_tensors(w.pos, w.carried, w.label, w.id, w.n_dev) for w in work]

        def reset(ctx):
            with torch.cuda.stream(stream):
                for w, sn in zip(work, snaps[k]):
                    for dst, src in zip(w.tensors(), sn.tensors()):
                        dst.copy_(src)
                # reading 1 GB evicts the 256 MB Infinity Cache without leaving dirty lines
                float(flush.sum())
            stream.synchronize()
            S.check(S.sph_state_set(ctx, *states[k][0]), "state_set")

        def replay(mode, ctx, profile, region=True):
            reset(ctx)
            S.check(S.sph_profile_enable(ctx, False), "profile")
            if mode == "local":
                # the automatic build method times both builds on the warm-up states
                # (synchronised builds, so every timing is read) and settles before
                # the timed steps, where it re-checks its choice every 64 builds
                S.check(S.sph_build_retune(ctx), "retune")
                for r in range(TUNE_BUILDS):
                    S.check(S.sph_celllist_build(ctx, parts[r % Wm]), "build")
                    stream.synchronize()
            for s in range(Wm):
                if mode == "local":
                    S.check(S.sph_celllist_build(ctx, parts[s]), "build")
                    S.check(S.sph_buffer_update_async(ctx, parts[s]), "update")
                else:
                    S.check(S.sph_buffer_update_fullscan_async(ctx, parts[s]), "fullscan")
            stream.synchronize()
            if profile:
                S.check(S.sph_profile_enable(ctx, True), "profile")
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            if k == "late" and region:
                REGIONS.begin()
            t0 = time.perf_counter()
            e0.record(stream)
            for s in range(Wm, Wm + K):
                if mode == "local":
                    S.sph_celllist_build(ctx, parts[s])
                    S.sph_buffer_update_async(ctx, parts[s])
                else:
                    S.sph_buffer_update_fullscan_async(ctx, parts[s])
            e1.record(stream)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            if k == "late" and region:
                REGIONS.end()
            ms = e0.elapsed_time(e1) / K
            rs, r = S.sph_last_result(ctx)
            S.check(r.status, f"{mode} replay")
            assert (r.n_before, r.n_after, r.n_generated, r.n_deleted) == nlist[k][-1], (mode, k)
            prof = None
            if profile:
                st, pms, pn = S.sph_profile_read(ctx, reset=True)
                S.check(S.sph_profile_enable(ctx, False), "profile")
                prof = {S.PHASES[i]: float(pms[i]) / max(1, int(pn[i])) for i in range(S.SPH_NPHASE) if pn[i] > 0}
            return ms, wall / K * 1e3, prof

        out = {}
        if k == "late":
            # a plain device copy of known size (the id array: 8 bytes x capacity) inside
            # a profiler region: the calibration of the HBM traffic counters
            src_ids, dst_ids = snaps[k][0].id, work[0].id
            torch.cuda.synchronize()
            REGIONS.begin()
            dst_ids.copy_(src_ids)
            torch.cuda.synchronize()
            REGIONS.end()
        out["ms_merged"], out["wall_merged"], _ = replay("local", dom.ctx, False)
        out["method"] = build_method(dom.ctx)
        out["ms_full"], _, _ = replay("fullscan", dom.ctx, False)
        out["ms_cells"], _, _ = replay("local", ctx_cells, False)
        # outside the profiler's regions: the profiled kernels stay those of the paths above
        out["ms_fixed"] = {m: replay("local", c, False, region=False)[0] for m, c in fixed.items()}
        if not args.no_profile_pass:
            _, _, out["prof_merged"] = replay("local", dom.ctx, True)
            _, _, out["prof_full"] = replay("fullscan", dom.ctx, True)
            _, _, out["prof_cells"] = replay("local", ctx_cells, True)
        out["n_mean"] = float(np.mean([x[0] for x in nlist[k][Wm:]]))
        out["g_mean"] = float(np.mean([x[2] for x in nlist[k][Wm:]]))
        out["d_mean"] = float(np.mean([x[3] for x in nlist[k][Wm:]]))
        out["work"], out["parts"] = work, parts
        return out

    res = {}
    for k in windows:
        res[k] = run_window(k)
        if k == "early":  # its working copies are not needed any more
            del res[k]["work"], res[k]["parts"]
            del snaps[k][:]
            torch.cuda.empty_cache()
    L = res["late"]
    # candidates of the local path on the first timed late state
    s0 = snaps["late"][Wm]
    n0 = int(s0.n_dev.item())
    cand = cover_candidates(np, S, wl, rots, [t.cpu().numpy() for t in s0.pos], n0)
    pm = L.get("prof_merged")
    # the method of the profiled replay (its timed steps run one method: no re-check falls there)
    meth = ("counting" if "scan" in pm else "bucketed") if pm else L["method"]["chosen"]
    pb = phase_bytes(wl.dim, int(L["n_mean"]), n_cells, cand, int(L["g_mean"]), int(L["d_mean"]), len(wl.carried),
                     meth)
    kernel_of = KERNEL_OF[meth]
    step_bytes = pb["build"] + pb["classify"] + pb["finalize"]
    ms = L["ms_merged"]
    n_mean = L["n_mean"]
    out = {"ms_per_step": round(ms, 5), "Mparticles_per_s": round(n_mean / (ms * 1e-3) / 1e6, 1),
           "n_particles": int(n_mean), "cells": n_cells, "candidates_per_update": cand,
           "events_per_step": {"generated": L["g_mean"], "deleted": L["d_mean"]},
           "timed_steps": f"{late + Wm}..{late + Wm + K - 1} (warm-up {late}..{late + Wm - 1})",
           "pct_hbm_peak_step": round(step_bytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS * 100, 2),
           "fullscan": {"ms_per_update": round(L["ms_full"], 5),
                        "Mparticles_per_s": round(n_mean / (L["ms_full"] * 1e-3) / 1e6, 1)},
           "speedup_step_vs_fullscan": round(L["ms_full"] / ms, 3)}
    pm, pf, pc = L.get("prof_merged"), L.get("prof_full"), L.get("prof_cells")
    if pm:
        dom_phase = max(pm, key=lambda k: pm[k])
        avg_ms = pm[dom_phase]
        achieved = pb[dom_phase] / (avg_ms * 1e-3) / 1e9
        kname = kernel_of.get(dom_phase, "k_" + dom_phase)
        out["roofline"] = {"bound": "hbm", "kernel": kname, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                           "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                           "traffic": measured_traffic(wl.name, kname), "avg_launch_us": round(avg_ms * 1e3, 2),
                           "algorithmic_bytes_per_launch": int(pb[dom_phase])}
        out["phases_us"] = {k: round(v * 1e3, 2) for k, v in pm.items()}
        out["phases_note"] = PHASES_NOTE[meth]
    out["build_method"] = L["method"]
    if pc:
        t_upd = pc.get("classify", 0.0) + pc.get("finalize", 0.0)
        t_full = pf["fullscan"] + pf.get("candidates", 0.0) + pf["finalize"] if pf else None
        out["local_update_only"] = {
            "ms": round(t_upd, 5), "Mparticles_per_s": round(n_mean / (t_upd * 1e-3) / 1e6, 1),
            "fullscan_update_ms": round(t_full, 5) if t_full else None,
            "speedup_vs_fullscan": round(t_full / t_upd, 2) if t_full else None,
            "what": "cover-cell walk's update (classify + finalize) with the cell list already built, against "
                    "the all-particle update (filter + candidates + finalize)"}
    out["cover_cell_walk"] = {"ms_per_step": round(L["ms_cells"], 5),
                              "Mparticles_per_s": round(n_mean / (L["ms_cells"] * 1e-3) / 1e6, 1),
                              "phases_us": {k: round(v * 1e3, 2) for k, v in pc.items()} if pc else None}
    if pf:
        out["fullscan_phases_us"] = {k: round(v * 1e3, 2) for k, v in pf.items()}
    E = res.get("early")
    if E is not None:
        out["early_window"] = {"timed_steps": f"{early + Wm}..{early + Wm + K - 1}",
                               "ms_per_step": round(E["ms_merged"], 5),
                               "Mparticles_per_s": round(E["n_mean"] / (E["ms_merged"] * 1e-3) / 1e6, 1),
                               "phases_us": {k: round(v * 1e3, 2) for k, v in E["prof_merged"].items()}
                               if E.get("prof_merged") else None,
                               "cover_cell_walk_ms": round(E["ms_cells"], 5),
                               "build_method": E["method"],
                               "fullscan_ms": round(E["ms_full"], 5)}
        out["drift_late_over_early"] = round(ms / E["ms_merged"], 3)
    log(f"{wl.name}: late step {ms * 1e3:.1f} us" + (f" (early {E['ms_merged'] * 1e3:.1f})" if E else "")
        + ", cover-cell walk "
        f"{L['ms_cells'] * 1e3:.1f} us, full-scan update {L['ms_full'] * 1e3:.1f} us; phases (us): "
        + ", ".join(f"{k} {v * 1e3:.1f}" for k, v in (pm or {}).items()))
    out["build_method"]["step_ms_each_method"] = {m: round(v, 5) for m, v in L["ms_fixed"].items()}
    if E is not None:
        out["early_window"]["build_method"]["step_ms_each_method"] = {m: round(v, 5) for m, v in E["ms_fixed"].items()}
    for c in fixed.values():
        S.sph_destroy(c)
    leg = {"out": out, "dom": dom, "ctx_cells": ctx_cells, "snaps": snaps["late"], "states": states["late"],
           "work": L["work"], "parts": L["parts"], "rots": rots, "stream": stream, "flush": flush}
    return leg


def close_leg(leg, S, torch):
    S.sph_destroy(leg["ctx_cells"])
    leg["dom"].close()
    leg.clear()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def bc_and_neighbor_legs(torch, np, S, leg, wl, K, Wm, args):
    """Boundary conditions and the solver's neighbour search on the pipe's states."""
    out = {}
    dom, snaps, states, work, parts, stream = (leg["dom"], leg["snaps"], leg["states"], leg["work"], leg["parts"],
                                               leg["stream"])

    def reset():
        with torch.cuda.stream(stream):
            for w, sn in zip(work, snaps):
                for dst, src in zip(w.tensors(), sn.tensors()):
                    dst.copy_(src)
            float(leg["flush"].sum())
        stream.synchronize()

    if not args.no_bc and wl.dim == 3:
        S.check(S.sph_set_fields(dom.ctx, [0, 1, 2], 4), "fields")
        S.check(S.sph_buffer_set_bc(dom.ctx, 1, S.SPH_BC_VELOCITY, profile=S.SPH_PROFILE_PARABOLIC_R, u=1.0,
                                    radius=0.05), "bc inlet")
        S.check(S.sph_buffer_set_bc(dom.ctx, 2, S.SPH_BC_PRESSURE, p_b=0.0, rho0=1000.0, c0=10.0), "bc outlet")
        reset()
        S.check(S.sph_profile_enable(dom.ctx, True), "profile")
        for s in range(Wm, Wm + K):
            S.check(S.sph_state_set(dom.ctx, *states[s]), "state_set")
            S.sph_celllist_build(dom.ctx, parts[s])
            S.check(S.sph_buffer_apply_bc(dom.ctx, parts[s]), "apply_bc")
        st_, pms, pn = S.sph_profile_read(dom.ctx, reset=True)
        S.check(S.sph_profile_enable(dom.ctx, False), "profile")
        bc_us = float(pms[S.PHASES.index("bc")]) / max(1, int(pn[S.PHASES.index("bc")])) * 1e3
        n_buf = int(sum(states[Wm][1][:2]))
        out["boundary_conditions"] = {
            "apply_bc_us": round(bc_us, 2), "buffer_particles": n_buf,
            "what": "velocity inlet (pipe profile) + pressure outlet (normal projection) on the labelled particles, "
                    "one kernel over the local cells"}
        log(f"apply_bc {bc_us:.1f} us on {n_buf} buffer particles")
    if not args.no_neighbor:
        dev = torch.device("cuda:0")
        counts = torch.empty(wl.capacity, dtype=torch.int32, device=dev)
        reset()
        S.check(S.sph_profile_enable(dom.ctx, True), "profile")
        n_nb = min(K, 5)
        for s in range(Wm, Wm + n_nb):
            S.check(S.sph_state_set(dom.ctx, *states[s]), "state_set")
            S.sph_celllist_build(dom.ctx, parts[s])
            S.check(S.sph_neighbor_count(dom.ctx, parts[s], wl.cell_size, counts.data_ptr()), "neighbor_count")
        st_, pms, pn = S.sph_profile_read(dom.ctx, reset=True)
        S.check(S.sph_profile_enable(dom.ctx, False), "profile")
        nb_us = float(pms[S.PHASES.index("neighbor")]) / max(1, int(pn[S.PHASES.index("neighbor")])) * 1e3
        n_last = int(snaps[Wm + n_nb - 1].n_dev.item())
        mean_nb = float(counts[:n_last].double().mean().item())
        out["neighbor_search"] = {
            "us": round(nb_us, 1), "radius": "cell size (2h = 2.6 dp)", "mean_neighbors": round(mean_nb, 2),
            "Mparticles_per_s": round(n_last / (nb_us * 1e-6) / 1e6, 1),
            "what": "neighbour counts over the library's cell list (FP32 distances, FP64 in the 2^-16 band)"}
        log(f"neighbor_count {nb_us:.1f} us, {mean_nb:.1f} neighbours per particle")
    return out


def sprinkler_leg(torch, np, S, W, Domain, steps: int = 40):
    """Rotating sprinkler (2-D) on a lawn of 2 M resting particles: per step the
    cell list, the update at the turning inlet, its velocity profile, the move of
    every particle with its own velocity and the turn of the buffer."""
    wl = W.sprinkler2d(n_background=2_000_000, capacity=2_200_000)
    d = Domain(wl.dim, wl.lo, wl.hi, wl.cell_size, wl.dp, wl.capacity, wl.pos, wl.carried, wl.label, wl.id,
               wl.n, wl.n, max_events=S.SPH_MAX_EVENTS_LIMIT)
    b = wl.buffers[0]
    d.define(b.kind, b.origin, rotation_of(S, b, 2), b.half, b.margin)
    d.set_fields([0, 1], 3)
    d.set_bc(1, S.SPH_BC_VELOCITY, profile=S.SPH_PROFILE_PARABOLIC_Y, u=wl.bc_u, radius=wl.bc_radius)
    S.check(d.identify(-1), "identify")
    m = W.rotation_z(wl.omega * wl.dt)
    stream = d.stream

    def step():
        # no host wait inside a step: the boundary conditions and the turn are
        # enqueued, and every slot of the arrays is moved (those past the live count
        # are never read)
        d.build()
        S.check(d.update_async(), "update")
        d.build()
        S.check(d.apply_bc_async(), "apply_bc")
        with torch.cuda.stream(stream):
            for c in range(2):
                d.pos[c].add_(d.carried[c] * wl.dt)
        d.build()
        S.check(d.rotate_async(1, (0.0, 0.0), m), "rotate")

    for _ in range(5):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / steps
    S.check(d.bc_status(), "boundary conditions and turns")
    S.check(d.result()[1].status, "update")
    # the library's kernel time per step, in a second run with per-launch events
    S.check(S.sph_profile_enable(d.ctx, True), "profile")
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    st, pms, pn = S.sph_profile_read(d.ctx, reset=True)
    ph = {S.PHASES[i]: float(pms[i]) / max(1, int(pn[i])) * 1e3 for i in range(S.SPH_NPHASE) if pn[i] > 0}
    per_step = sum(float(pms[i]) for i in range(S.SPH_NPHASE)) / steps * 1e3
    n = d.n()
    d.close()
    log(f"sprinkler: N = {n}, rotate {ph.get('rotate', 0):.1f} us + cover {ph.get('cover', 0):.1f} us, "
        f"bc {ph.get('bc', 0):.1f} us, "
        f"wall {wall * 1e3:.3f} ms/step, library kernels {per_step:.1f} us/step")
    return {"n_particles": n, "steps": steps, "rotate_us": round(ph.get("rotate", 0.0), 2),
            "turned_cover_us": round(ph.get("cover", 0.0), 2),
            "apply_bc_us": round(ph.get("bc", 0.0), 2), "phases_us": {k: round(v, 2) for k, v in ph.items()},
            "wall_ms_per_step": round(wall * 1e3, 3), "library_kernels_us_per_step": round(per_step, 2),
            "wall_over_kernels": round(wall * 1e6 / per_step, 2) if per_step > 0 else None}


def batch_leg(torch, np, S, W, Domain, steps: int, warmup: int, fixed=None):
    """64 hub-and-spoke domains: batched step (autotuned launch mode, graph replay)
    against a per-domain loop of plain launches, on the same prepared states.
    fixed = (mode, particles per count block, runs per classify workgroup) skips
    the autotuner."""
    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    wls = W.hub_batch()
    log(f"batch: {len(wls)} domains, N = {sum(w.n for w in wls)}, generated in {time.perf_counter() - t0:.1f} s")
    doms = []
    for wl in wls:
        dims = np.ceil((np.array(wl.hi[: wl.dim]) - np.array(wl.lo[: wl.dim])) / wl.cell_size)
        blog2 = 3 if wl.dim == 3 and np.prod(dims) > 2 * wl.n else 0
        d = Domain(wl.dim, wl.lo, wl.hi, wl.cell_size, wl.dp, wl.capacity, wl.pos, wl.carried, wl.label, wl.id,
                   wl.n, wl.n, max_events=S.SPH_MAX_EVENTS_LIMIT, brick_log2=blog2)
        for b in wl.buffers:
            d.define(b.kind, b.origin, rotation_of(S, b, wl.dim), b.half, b.margin)
        if blog2:
            d.fit()
        S.check(d.identify(-1), "identify")
        doms.append(d)
    stream = doms[0].stream
    n_snap = warmup + steps
    snaps, states, finals = [], [], []
    gen = torch.Generator(device=dev)
    for s in range(n_snap):
        states.append([S.sph_state_get(d.ctx)[1:] for d in doms])
        snaps.append([Snapshot(d) for d in doms])
        for d in doms:
            d.build()
            S.check(d.update_async(), "update")
        finals.append([d.result()[1].n_after for d in doms])
        for k, (wl, d) in enumerate(zip(wls, doms)):
            n = int(d.n_dev.item())
            gen.manual_seed(wl.seed_noise + s)
            with torch.cuda.stream(stream):
                p = [t[:n] for t in d.pos]
                noise = torch.randn((wl.dim, n), generator=gen, device=dev, dtype=torch.float32)
                u = wl.velocity(torch, p, s, noise)
                for c in range(wl.dim):
                    p[c].add_(u[c] * wl.dt)
    stream.synchronize()
    work = [[Snapshot(d) for d in doms] for _ in range(n_snap)]
    parts = [[S.particles_from_tensors(w.pos, w.carried, w.label, w.id, w.n_dev) for w in ws] for ws in work]
    flush = torch.ones(1 << 28, dtype=torch.float32, device=dev)
    bstream = torch.cuda.Stream()

    def reset():
        with torch.cuda.stream(stream):
            for ws, ss in zip(work, snaps):
                for w, sn in zip(ws, ss):
                    for dst, src_ in zip(w.tensors(), sn.tensors()):
                        dst.copy_(src_)
            float(flush.sum())
        torch.cuda.synchronize()
        for d, (nid, nl) in zip(doms, states[0]):
            S.check(S.sph_state_set(d.ctx, nid, nl), "state_set")

    def check_final():
        for d, expect in zip(doms, finals[-1]):
            st, r = S.sph_last_result(d.ctx)
            S.check(r.status, "batch leg")
            assert r.n_after == expect, (r.n_after, expect)

    # per-domain loop of plain launches
    reset()
    for s in range(warmup):
        for d, p in zip(doms, parts[s]):
            S.sph_celllist_build(d.ctx, p)
            S.sph_buffer_update_async(d.ctx, p)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for s in range(warmup, n_snap):
        for d, p in zip(doms, parts[s]):
            S.sph_celllist_build(d.ctx, p)
            S.sph_buffer_update_async(d.ctx, p)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_loop = e0.elapsed_time(e1) / steps
    check_final()

    # batched: one batch per prepared state; tune on the first, capture all, then replay
    batches = []
    for s in range(n_snap):
        st, b = S.sph_batch_create([d.ctx for d in doms], parts[s], bstream.cuda_stream)
        S.check(st, "batch_create")
        batches.append(b)
    reset()
    if fixed:
        mode, ppb, rpb = fixed
    else:
        st, mode, ppb, ms_tuned = S.sph_batch_tune(batches[0], 3, None)
        S.check(st, "tune")
        st, mode, ppb, rpb = S.sph_batch_get_config(batches[0])
        S.check(st, "config")
    for b in batches:
        S.check(S.sph_batch_set_mode(b, mode), "mode")
        S.check(S.sph_batch_set_count_block(b, ppb), "ppb")
        S.check(S.sph_batch_set_gather(b, rpb), "gather")
    reset()
    for b in batches:                      # first step of a graph-mode batch captures its graph
        S.check(S.sph_batch_step(b), "capture")
    torch.cuda.synchronize()
    reset()
    for s in range(warmup):
        S.check(S.sph_batch_step(batches[s]), "batch step")
    torch.cuda.synchronize()
    e0.record(bstream)
    for s in range(warmup, n_snap):
        S.sph_batch_step(batches[s])
    e1.record(bstream)
    torch.cuda.synchronize()
    ms_batch = e0.elapsed_time(e1) / steps
    check_final()
    # per-launch times of the batched phases (launch mode, same states)
    reset()
    for s in range(warmup):
        S.check(S.sph_batch_set_mode(batches[s], S.SPH_BATCH_KERNELS), "mode")
        S.check(S.sph_batch_step(batches[s]), "batch step")
    for s in range(warmup, n_snap):
        S.check(S.sph_batch_set_mode(batches[s], S.SPH_BATCH_KERNELS), "mode")
        S.check(S.sph_batch_profile_enable(batches[s], True), "profile")
        S.check(S.sph_batch_step(batches[s]), "batch step")
    torch.cuda.synchronize()
    tot = np.zeros(5)
    cnt = np.zeros(5, dtype=np.int64)
    for s in range(warmup, n_snap):
        st, pms, pn = S.sph_batch_profile_read(batches[s])
        tot += pms
        cnt += pn
    ph = {S.BATCH_PHASES[i]: tot[i] / max(1, cnt[i]) for i in range(5) if cnt[i] > 0}
    check_final()
    n_total = sum(w.n for w in wls)
    count_bytes = sum(4 * w.dim * w.n for w in wls)
    step_bytes = sum((4 * w.dim + 4) * w.n for w in wls)
    roof = None
    if "count" in ph:
        ach = count_bytes / (ph["count"] * 1e-3) / 1e9
        roof = {"bound": "hbm", "kernel": "kb_count", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": None,
                "avg_launch_us": round(ph["count"] * 1e3, 2), "algorithmic_bytes_per_launch": int(count_bytes)}
    for b in batches:
        S.sph_batch_destroy(b)
    for d in doms:
        d.close()
    log(f"batch: loop {ms_loop * 1e3:.0f} us/step, batched {ms_batch * 1e3:.0f} us/step "
        f"(mode {'graph' if mode == 1 else 'kernels'}, {ppb} particles per count block, {rpb} runs per "
        f"classify workgroup); phases (us): "
        + ", ".join(f"{k} {v * 1e3:.1f}" for k, v in ph.items()))
    return {"domains": len(wls), "n_particles": n_total, "buffers": sum(len(w.buffers) for w in wls),
            "ms_per_step_batched": round(ms_batch, 4), "ms_per_step_loop": round(ms_loop, 4),
            "speedup_batched_vs_loop": round(ms_loop / ms_batch, 2),
            "Mparticles_per_s_batched": round(n_total / (ms_batch * 1e-3) / 1e6, 1),
            "Mparticles_per_s_loop": round(n_total / (ms_loop * 1e-3) / 1e6, 1),
            "pct_hbm_peak_build": round(step_bytes / (ms_batch * 1e-3) / 1e9 / HBM_PEAK_GBS * 100, 2),
            "phases_us": {k: round(v * 1e3, 2) for k, v in ph.items()}, "roofline": roof,
            "tuned": {"mode": "graph" if mode == 1 else "kernels", "particles_per_count_block": ppb,
                      "runs_per_classify_workgroup": rpb}}


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def cpu_baseline(np, leg, wl, Wm, budget_s: float):
    """The FP64 oracle on this host's cores, on the first timed state of the
    headline workload: brute force on one thread and on all threads, and the
    paper's local-cell method (cell list given) on all threads."""
    import oracle
    sn, nid = leg["snaps"][Wm], int(leg["states"][Wm][0])
    nl_in = [int(x) for x in leg["states"][Wm][1][: len(wl.buffers)]]
    pos = [t.cpu().numpy() for t in sn.pos]
    car = [t.cpu().numpy() for t in sn.carried]
    lab = sn.label.cpu().numpy()
    ids = sn.id.cpu().numpy()
    n0 = int(sn.n_dev.item())
    ob = []
    for b in wl.buffers:
        q = oracle.rotation_2d(b.angle) if wl.dim == 2 else oracle.rotation_from_direction(b.direction)
        ob.append(oracle.Buffer(b.kind, b.origin, q, b.half, b.margin))

    def fresh():
        return oracle.State(wl.dim, [a.copy() for a in pos], [a.copy() for a in car], lab.copy(), ids.copy(), n0, nid)

    def timed(fn, seconds, max_n=50):
        times = []
        t_start = time.perf_counter()
        while not times or (time.perf_counter() - t_start < seconds and len(times) < max_n):
            st = fresh()
            t0 = time.perf_counter()
            res = fn(st)
            times.append(time.perf_counter() - t0)
            assert res.status == 0, res.status
        return float(np.median(times)), len(times)

    n_all = oracle.set_threads(0)
    oracle.set_threads(1)
    t1, k1 = timed(lambda st: oracle.update(ob, st), 0.35 * budget_s)
    oracle.set_threads(n_all)
    ta, ka = timed(lambda st: oracle.update(ob, st), 0.3 * budget_s)
    dims = [int(math.ceil((wl.hi[c] - wl.lo[c]) / wl.cell_size)) for c in range(wl.dim)]
    lo32 = np.float32(wl.lo[: wl.dim])
    inv = np.float32(1.0 / wl.cell_size)
    t0 = time.perf_counter()
    start, idx = oracle.cell_list(wl.dim, lo32, inv, dims, pos[0][:n0], pos[1][:n0], pos[2][:n0] if wl.dim == 3 else None)
    t_cells = time.perf_counter() - t0
    tl, kl = timed(lambda st: oracle.update_local(ob, st, lo32, inv, dims, start, idx, nl_in), 0.2 * budget_s)
    del start, idx
    log(f"cpu oracle ({n_all} threads, {cpu_model()}): brute 1T {t1 * 1e3:.0f} ms, brute {n_all}T "
        f"{ta * 1e3:.0f} ms, local-cell {tl * 1e3:.1f} ms (+ cell list {t_cells * 1e3:.0f} ms, 1T)")
    return {"value": round(n0 / ta / 1e6, 2), "unit": "Mparticles/s", "cores": n_all, "kind": "oracle",
            "sample": f"{ka} FP64 brute-force oracle updates of the first timed state of {wl.name} (N = {n0}) on "
                      f"{n_all} threads, median {ta * 1e3:.0f} ms",
            "cpu_model": cpu_model(), "os_cpu_count": os.cpu_count(),
            "one_thread": {"value": round(n0 / t1 / 1e6, 2), "median_ms": round(t1 * 1e3, 1), "updates": k1},
            "all_threads": {"value": round(n0 / ta / 1e6, 2), "median_ms": round(ta * 1e3, 1), "updates": ka},
            "local_cell_all_threads": {"value": round(n0 / tl / 1e6, 2), "median_ms": round(tl * 1e3, 2),
                                       "updates": kl, "cell_list_build_ms_one_thread": round(t_cells * 1e3, 1),
                                       "what": "the paper's method on the CPU: candidates only from the cells "
                                               "near each check region of a dense FP32 cell list (given)"}}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="tree3d", choices=sorted(DESCRIPTION))
    ap.add_argument("--late", type=int, default=None, help="first state of the timed (late) window")
    ap.add_argument("--early", type=int, default=5, help="first state of the early window")
    ap.add_argument("--late-only", action="store_true", help="time the late window only (no drift)")
    ap.add_argument("--cpu-seconds", type=float, default=24.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile-pass", action="store_true")
    ap.add_argument("--no-pipe", action="store_true", help="skip the 3-D pipe leg")
    ap.add_argument("--no-batch", action="store_true", help="skip the 64-domain batched leg")
    ap.add_argument("--no-bc", action="store_true", help="skip the boundary-condition leg")
    ap.add_argument("--no-sprinkler", action="store_true", help="skip the rotating-sprinkler leg")
    ap.add_argument("--no-neighbor", action="store_true", help="skip the neighbour-search leg")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1",
                          "n_gpus_requested": args.gpus}), flush=True)
        return 2

    import numpy as np
    import torch

    import workloads as W
    from paper_2406_16786_amd import sphbuf as S
    from paper_2406_16786_amd.domain import Domain

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    K, Wm = args.steps, args.warmup
    t_all = time.perf_counter()
    late = args.late if args.late is not None else LATE_START[args.workload]

    t0 = time.perf_counter()
    wl = make_workload(args.workload)
    log(f"workload {wl.name}: N = {wl.n}, dim {wl.dim}, capacity {wl.capacity} "
        f"(generated in {time.perf_counter() - t0:.1f} s)")
    leg = single_leg(torch, np, S, W, Domain, wl, K, Wm, late, args.early, args)
    h = leg["out"]
    out = {
        "metric": METRIC,
        "value": h["Mparticles_per_s"],
        "unit": "Mparticles/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": Wm,
        "ms_per_step": h["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 (f64 recheck in the guard band)",
        "data": "synthetic",
        "config": {"workload": f"{wl.name}: {DESCRIPTION[wl.name]}", "n_particles": h["n_particles"],
                   "dim": wl.dim, "buffers": len(wl.buffers), "cells": h["cells"],
                   "candidates_per_update": h["candidates_per_update"], "events_per_step": h["events_per_step"],
                   "timed_steps": h["timed_steps"],
                   "path": "merged step: cell-list build (counting or bucketed sort, whichever the context "
                           "timed faster; build_method) whose count pass lists the cover cells' candidates; their "
                           "exact tests beside the build's scatter; finalize"},
        "roofline": h.get("roofline"),
    }
    for k, v in h.items():
        if k not in ("ms_per_step", "Mparticles_per_s", "n_particles", "cells", "candidates_per_update",
                     "events_per_step", "timed_steps", "roofline"):
            out[k] = v
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(np, leg, wl, Wm, args.cpu_seconds)
    close_leg(leg, S, torch)
    del wl

    out["legs"] = {}
    if not args.no_pipe and args.workload != "pipe3d":
        t0 = time.perf_counter()
        wp = make_workload("pipe3d")
        log(f"workload pipe3d: N = {wp.n} (generated in {time.perf_counter() - t0:.1f} s)")
        lp = single_leg(torch, np, S, W, Domain, wp, K, Wm, LATE_START["pipe3d"], args.early, args)
        o = lp["out"]
        o["workload"] = f"pipe3d: {DESCRIPTION['pipe3d']}"
        out["legs"]["pipe3d"] = o
        out.update(bc_and_neighbor_legs(torch, np, S, lp, wp, K, Wm, args))
        close_leg(lp, S, torch)
        del wp
    if not args.no_sprinkler:
        out["sprinkler"] = sprinkler_leg(torch, np, S, W, Domain)
    if not args.no_batch:
        out["batched"] = batch_leg(torch, np, S, W, Domain, max(4, K // 2), max(1, Wm // 2))
    log(f"total {time.perf_counter() - t_all:.1f} s")
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())

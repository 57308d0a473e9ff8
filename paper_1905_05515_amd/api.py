"""Python binding of libtpc.so: torch tensors for device memory and streams,
argument marshalling to the C ABI.  Every step runs in the library's HIP
kernels; nothing here computes the method."""
from __future__ import annotations

import ctypes as C
import math
from dataclasses import dataclass, field

import numpy as np
import torch

from . import _lib as L
from .layout import SECTOR_DTYPE, grid_layout

MODES = {"staged": 0, "per_sector": 1, "persistent": 2}

# clusters per bin of the grid when no layout is given: small bins keep the
# window searches short (the tracks do not depend on this choice)
DEFAULT_OCCUPANCY = 0.25
# occupancies the autotuner tries
TUNE_OCCUPANCIES = (0.0625, 0.125, 0.25, 0.5, 1.0)


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def params_struct(prm: dict) -> L.Params:
    p = L.Params()
    for name, _ in L.Params._fields_:
        setattr(p, name, prm[name])
    return p


class Context:
    """A library context bound to one device."""

    def __init__(self, device: int = 0):
        self.device = device
        h = C.c_void_p()
        L.check(L.lib().tpc_context_create(C.byref(h), device), "tpc_context_create")
        self.handle = h
        self.tuned = {}     # autotuned occupancy per (sectors, clusters, mode)

    def close(self):
        if self.handle:
            L.lib().tpc_context_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclass
class Event:
    """Device buffers of one tracking problem (inputs, every output and the
    workspace).  Sizes: grid and links n_clusters; starts and tracklets
    start_capacity (n_clusters // 3 by default: a chain start needs three
    distinct hits); tracks up to start_capacity, their hits up to
    n_clusters."""
    problem: L.Problem
    keep: list = field(default_factory=list)
    t: dict = field(default_factory=dict)
    n_rows: int = 152
    start_capacity: int = 0
    ws_bytes: int = 0


def make_event(row, y, z, sector_offsets, sector_range, row_x, prm: dict, device="cuda",
               layout=None, occupancy=None, start_capacity=None, track_capacity=None,
               track_hit_capacity=None, sector_side=None) -> Event:
    """Copy an event to the device and allocate all outputs."""
    n_rows = int(np.asarray(row_x).shape[0])
    if occupancy is None:
        occupancy = DEFAULT_OCCUPANCY
    if layout is None:
        layout = grid_layout(sector_offsets, sector_range, n_rows=n_rows, occupancy=occupancy,
                             sides=sector_side)
    tab, n_bins = layout
    tab = np.ascontiguousarray(tab, dtype=SECTOR_DTYPE)
    n = int(np.asarray(row).shape[0])
    cap = int(start_capacity if start_capacity is not None else max(n // 3, 1))
    tcap = int(track_capacity if track_capacity is not None else cap)
    hcap = int(track_hit_capacity if track_hit_capacity is not None else max(n, 1))
    dev = torch.device(device)

    def to_dev(a, dt):
        return torch.as_tensor(np.ascontiguousarray(a), dtype=dt).to(dev)

    t = {}
    t["row"] = to_dev(row, torch.uint8)
    t["y"] = to_dev(y, torch.float32)
    t["z"] = to_dev(z, torch.float32)
    t["row_x"] = to_dev(np.asarray(row_x, np.float32), torch.float32)
    h_sec = torch.from_numpy(tab.view(np.uint8).copy())
    t["h_sectors"] = h_sec
    t["d_sectors"] = h_sec.to(dev)
    i32 = dict(dtype=torch.int32, device=dev)
    f32 = dict(dtype=torch.float32, device=dev)
    nn = max(n, 1)
    t["bin_start"] = torch.empty(n_bins + 1, **i32)
    t["yg"] = torch.empty(nn, **f32)
    t["zg"] = torch.empty(nn, **f32)
    t["idg"] = torch.empty(nn, **i32)
    for k in ("up0", "down0", "up", "down"):
        t[k] = torch.empty(nn, **i32)
    t["starts"] = torch.empty(cap, **i32)
    t["t_start"] = torch.empty(cap, **i32)
    t["t_hits"] = torch.empty(cap * n_rows, **i32)
    t["t_nhits"] = torch.empty(cap, **i32)
    t["t_rin"] = torch.empty(cap, **i32)
    t["t_par"] = torch.empty(cap * 5, **f32)
    t["t_cov"] = torch.empty(cap * 15, **f32)
    t["t_chi2"] = torch.empty(cap, **f32)
    t["trk_off"] = torch.empty(tcap + 1, **i32)
    t["trk_hits"] = torch.empty(hcap, **i32)
    # the hits' rows and coordinates in track order (written by the selection)
    t["trk_row"] = torch.empty(hcap, dtype=torch.uint8, device=dev)
    t["trk_y"] = torch.empty(hcap, dtype=torch.float32, device=dev)
    t["trk_z"] = torch.empty(hcap, dtype=torch.float32, device=dev)
    t["trk_tracklet"] = torch.empty(max(tcap, 1), **i32)
    t["trk_side"] = torch.empty(max(tcap, 1), dtype=torch.int8, device=dev)
    prob = L.Problem()
    prob.n_sectors = tab.shape[0]
    prob.n_rows = n_rows
    prob.n_clusters = n
    prob.n_bins = n_bins
    prob.h_sectors = C.c_void_p(h_sec.data_ptr())
    prob.d_sectors = C.c_void_p(t["d_sectors"].data_ptr())
    prob.d_row_x = C.c_void_p(t["row_x"].data_ptr())
    prob.params = params_struct(prm)
    nbytes = C.c_size_t()
    L.check(L.lib().tpc_workspace_size(C.byref(prob), cap, C.byref(nbytes)), "tpc_workspace_size")
    t["ws"] = torch.empty(max(int(nbytes.value), 256), dtype=torch.uint8, device=dev)
    ev = Event(problem=prob, t=t, n_rows=n_rows, start_capacity=cap, ws_bytes=int(nbytes.value))
    ev.track_capacity = tcap
    ev.track_hit_capacity = hcap
    ev.layout = (tab, n_bins)
    ev.layout_args = (np.asarray(sector_offsets), np.asarray(sector_range), sector_side)
    ev.occupancy = occupancy
    return ev


def relayout(ev: Event, occupancy: float = None, layout=None):
    """Give the event another bin grid (by occupancy, or an explicit layout
    table): reallocates the bin starts and the workspace."""
    offs, rng, sides = ev.layout_args
    if layout is None:
        layout = grid_layout(offs, rng, n_rows=ev.n_rows, occupancy=occupancy, sides=sides)
    tab, n_bins = layout
    tab = np.ascontiguousarray(tab, dtype=SECTOR_DTYPE)
    t = ev.t
    dev = t["y"].device
    h_sec = torch.from_numpy(tab.view(np.uint8).copy())
    t["h_sectors"] = h_sec
    t["d_sectors"] = h_sec.to(dev)
    t["bin_start"] = torch.empty(n_bins + 1, dtype=torch.int32, device=dev)
    prob = ev.problem
    prob.n_bins = n_bins
    prob.h_sectors = C.c_void_p(h_sec.data_ptr())
    prob.d_sectors = C.c_void_p(t["d_sectors"].data_ptr())
    nbytes = C.c_size_t()
    L.check(L.lib().tpc_workspace_size(C.byref(prob), ev.start_capacity, C.byref(nbytes)),
            "tpc_workspace_size")
    t["ws"] = torch.empty(max(int(nbytes.value), 256), dtype=torch.uint8, device=dev)
    ev.ws_bytes = int(nbytes.value)
    ev.layout = (tab, n_bins)
    ev.occupancy = occupancy


TUNING_FIELDS = ("tracklet_form", "neighbour_block", "persistent_scale",
                 "persistent_blocks_per_cu")


def get_tuning(ctx: "Context") -> dict:
    """The context's launch shapes (0: the library's automatic choice)."""
    t = L.Tuning()
    L.check(L.lib().tpc_context_get_tuning(ctx.handle, C.byref(t)), "tpc_context_get_tuning")
    return {k: int(getattr(t, k)) for k in TUNING_FIELDS}


def set_tuning(ctx: "Context", **kw):
    """Set launch shapes of the context (fields of TUNING_FIELDS; the others
    keep their values).  No output depends on them."""
    cur = get_tuning(ctx)
    for k, v in kw.items():
        if k not in cur:
            raise KeyError(k)
        cur[k] = int(v)
    L.check(L.lib().tpc_context_set_tuning(ctx.handle, C.byref(L.Tuning(**cur))),
            "tpc_context_set_tuning")


# launch shapes the shape tuner tries, per tracking form, one field at a time
TUNE_SHAPES = {
    "staged": (("tracklet_form", (0, 1, 2, 3)), ("neighbour_block", (256, 128, 64))),
    "per_sector": (("tracklet_form", (0, 1, 2, 3)), ("neighbour_block", (256, 128, 64))),
    "persistent": (("persistent_scale", (0, 1, 2, 4, 8)), ("persistent_blocks_per_cu", (0, 2, 1)),
                   ("tracklet_form", (0,))),
}


def _time_batch(ctx, ev, mode, reps, s):
    with torch.cuda.stream(s):
        track_batch(ctx, ev, mode=mode, stream=s)          # warm
        ms = []
        for _ in range(reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(s)
            track_batch(ctx, ev, mode=mode, stream=s)
            b.record(s)
            b.synchronize()
            ms.append(a.elapsed_time(b))
    return sorted(ms)[len(ms) // 2]


def _track_digest(ev, s):
    """The track list on the host (offsets, hits) for the invariance check."""
    s.synchronize()
    st = get_status(ev, s)
    nt, nh = int(st["n_tracks"]), int(st["n_track_hits"])
    return (ev.t["trk_off"][:nt + 1].cpu().numpy().tobytes(),
            ev.t["trk_hits"][:nh].cpu().numpy().tobytes())


def autotune_shapes(ctx: "Context", ev: Event, mode: str = "staged", reps: int = 3,
                    stream=None):
    """Time the tracking chain for the launch shapes of TUNE_SHAPES[mode],
    one field at a time (each field keeps its fastest value before the next
    is tried), check that every shape gives the same tracks (raises
    otherwise) and leave the fastest shapes set.  Returns (shapes, {(field,
    value): ms})."""
    s = stream if stream is not None else torch.cuda.current_stream()
    times = {}
    ref = None
    for field_, values in TUNE_SHAPES[mode]:
        best_v, best_ms = None, None
        for v in values:
            set_tuning(ctx, **{field_: v})
            ms = _time_batch(ctx, ev, mode, reps, s)
            dig = _track_digest(ev, s)
            if ref is None:
                ref = dig
            elif dig != ref:
                raise RuntimeError(f"tracks differ with {field_}={v}")
            times[(field_, v)] = ms
            if best_ms is None or ms < best_ms:
                best_v, best_ms = v, ms
        set_tuning(ctx, **{field_: best_v})
    return get_tuning(ctx), times


def autotune(ctx: "Context", ev: Event, mode: str = "staged", candidates=TUNE_OCCUPANCIES,
             reps: int = 3, stream=None):
    """Time the tracking chain of this event for each bin occupancy and keep
    the fastest layout.  The tracks do not depend on the layout, so the
    choice only moves time.  Returns (best occupancy, {occupancy: ms}); the
    choice is remembered in the context per event shape."""
    s = stream if stream is not None else torch.cuda.current_stream()
    times = {}
    for occ in candidates:
        relayout(ev, occ)
        with torch.cuda.stream(s):
            track_batch(ctx, ev, mode=mode, stream=s)          # warm
            ms = []
            for _ in range(reps):
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record(s)
                track_batch(ctx, ev, mode=mode, stream=s)
                b.record(s)
                b.synchronize()
                ms.append(a.elapsed_time(b))
        times[occ] = sorted(ms)[len(ms) // 2]
    best = min(times, key=lambda k: (times[k], k))
    relayout(ev, best)
    ctx.tuned[(ev.problem.n_sectors, ev.problem.n_clusters, mode)] = best
    return best, times


def _clusters(ev):
    t = ev.t
    return L.Clusters(_ptr(t["row"]), _ptr(t["y"]), _ptr(t["z"]))


def _grid(ev):
    t = ev.t
    return L.Grid(_ptr(t["bin_start"]), _ptr(t["yg"]), _ptr(t["zg"]), _ptr(t["idg"]))


def _links(ev):
    t = ev.t
    return L.Links(_ptr(t["up0"]), _ptr(t["down0"]), _ptr(t["up"]), _ptr(t["down"]))


def _starts(ev):
    return L.Starts(_ptr(ev.t["starts"]), ev.start_capacity)


def _tracklets(ev):
    t = ev.t
    return L.Tracklets(_ptr(t["t_start"]), _ptr(t["t_hits"]), _ptr(t["t_nhits"]), _ptr(t["t_rin"]),
                       _ptr(t["t_par"]), _ptr(t["t_cov"]), _ptr(t["t_chi2"]), ev.start_capacity)


def _tracks(ev):
    t = ev.t
    return L.Tracks(_ptr(t["trk_off"]), _ptr(t["trk_hits"]), _ptr(t["trk_tracklet"]),
                    _ptr(t["trk_side"]), ev.track_capacity, ev.track_hit_capacity,
                    _ptr(t["trk_row"]), _ptr(t["trk_y"]), _ptr(t["trk_z"]))


def build_grid(ctx: Context, ev: Event, stream=None):
    L.check(L.lib().tpc_build_grid(ctx.handle, C.byref(ev.problem), _clusters(ev), _grid(ev),
                                   _ptr(ev.t["ws"]), ev.ws_bytes, _stream(stream)),
            "tpc_build_grid")


def find_neighbours(ctx: Context, ev: Event, stream=None):
    L.check(L.lib().tpc_find_neighbours(ctx.handle, C.byref(ev.problem), _grid(ev), _links(ev),
                                        _starts(ev), _ptr(ev.t["ws"]), ev.ws_bytes,
                                        _stream(stream)), "tpc_find_neighbours")


def construct_tracklets(ctx: Context, ev: Event, stream=None):
    L.check(L.lib().tpc_construct_tracklets(ctx.handle, C.byref(ev.problem), _grid(ev),
                                            _links(ev), _starts(ev), _tracklets(ev),
                                            _ptr(ev.t["ws"]), ev.ws_bytes, _stream(stream)),
            "tpc_construct_tracklets")


def select_tracks(ctx: Context, ev: Event, stream=None):
    L.check(L.lib().tpc_select_tracks(ctx.handle, C.byref(ev.problem), _grid(ev),
                                      _tracklets(ev), _tracks(ev), _ptr(ev.t["ws"]), ev.ws_bytes,
                                      _stream(stream)), "tpc_select_tracks")


def track_batch(ctx: Context, ev: Event, mode="staged", use_graph=False, stream=None):
    L.check(L.lib().tpc_track_batch(ctx.handle, C.byref(ev.problem), _clusters(ev), _grid(ev),
                                    _links(ev), _starts(ev), _tracklets(ev), _tracks(ev),
                                    _ptr(ev.t["ws"]), ev.ws_bytes, MODES[mode],
                                    1 if use_graph else 0, _stream(stream)), "tpc_track_batch")


def attach_clusters(ctx: Context, ev: Event, radius: float = 1.5, pt_good: float = 0.05,
                    stream=None):
    """Track-based cluster attachment of the event's found tracks (after
    the tracking calls): returns device tensors (track int32, state uint8)
    per cluster id; state bits 1 attached, 2 adjacent, 4 protected, 8
    removed."""
    n = ev.problem.n_clusters
    dev = ev.t["row"].device
    need = C.c_size_t(0)
    L.check(L.lib().tpc_attach_workspace_size(C.byref(ev.problem), C.byref(need)),
            "tpc_attach_workspace_size")
    ws = ev.t.get("attach_ws")
    if ws is None or ws.numel() < need.value:
        ws = torch.empty(max(need.value, 1), dtype=torch.uint8, device=dev)
        ev.t["attach_ws"] = ws
    track = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
    state = torch.empty(max(n, 1), dtype=torch.uint8, device=dev)
    L.check(L.lib().tpc_attach_clusters(ctx.handle, C.byref(ev.problem), _clusters(ev), _grid(ev),
                                        _tracklets(ev), _tracks(ev), status_count_ptr(ev),
                                        float(radius), float(pt_good), _ptr(track), _ptr(state),
                                        _ptr(ws), ws.numel(), _stream(stream)),
            "tpc_attach_clusters")
    return track[:n], state[:n]


MERGE_WINDOWS = (3.0, 2.0, 0.1, 0.02, 2.0)   # y, z [cm], sin(phi), tan(lambda), q/pT


def merge_cuts(sectors_per_side: int = 18, windows=MERGE_WINDOWS) -> "L.MergeCuts":
    """Cuts of the sector-track merging: the sector width is the full turn
    over sectors_per_side; cos, sin and the inverse windows in float32."""
    w = math.radians(360.0 / sectors_per_side)
    iw = np.float32(1.0) / np.asarray(windows, np.float32)
    cuts = L.MergeCuts()
    cuts.sectors_per_side = int(sectors_per_side)
    cuts.cos_width = float(np.float32(math.cos(w)))
    cuts.sin_width = float(np.float32(math.sin(w)))
    for i in range(5):
        cuts.inv_window[i] = float(iw[i])
    return cuts


def merge_sector_tracks(ctx: Context, ev: Event, sectors_per_side: int = 18,
                        windows=MERGE_WINDOWS, stream=None):
    """Sector-track merging of the event's found tracks (after the tracking
    calls): returns device tensors (link_up, link_dn, group) of
    tracks.capacity entries; the first n_tracks of them are written."""
    dev = ev.t["row"].device
    cap = ev.track_capacity
    need = C.c_size_t(0)
    L.check(L.lib().tpc_merge_workspace_size(C.byref(ev.problem), cap, C.byref(need)),
            "tpc_merge_workspace_size")
    ws = ev.t.get("merge_ws")
    if ws is None or ws.numel() < need.value:
        ws = torch.empty(max(need.value, 1), dtype=torch.uint8, device=dev)
        ev.t["merge_ws"] = ws
    out = [torch.empty(max(cap, 1), dtype=torch.int32, device=dev) for _ in range(3)]
    L.check(L.lib().tpc_merge_sector_tracks(ctx.handle, C.byref(ev.problem), _tracklets(ev),
                                            _tracks(ev), status_count_ptr(ev),
                                            merge_cuts(sectors_per_side, windows),
                                            *[_ptr(o) for o in out], _ptr(ws), ws.numel(),
                                            _stream(stream)),
            "tpc_merge_sector_tracks")
    return tuple(out)


def fit_merged_tracks(ctx: Context, ev: Event, links, sectors_per_side: int = 18,
                      n_pass: int = 3, cov_scale: float = 100.0, stream=None):
    """Full-track fit of the merged sector tracks (after merge_sector_tracks,
    whose (link_up, link_dn, group) are `links`): dict of device tensors of
    tracks.capacity entries (par_in, par_out [cap, 5], cov_out [cap, 15],
    chi2, n_hits, n_members, status); the first n_tracks are written, group
    leaders carry the fit."""
    dev = ev.t["row"].device
    cap = max(ev.track_capacity, 1)
    f32 = dict(dtype=torch.float32, device=dev)
    i32 = dict(dtype=torch.int32, device=dev)
    out = dict(par_in=torch.empty(cap, 5, **f32), par_out=torch.empty(cap, 5, **f32),
               cov_out=torch.empty(cap, 15, **f32), chi2=torch.empty(cap, **f32),
               n_hits=torch.empty(cap, **i32), n_members=torch.empty(cap, **i32),
               status=torch.empty(cap, **i32))
    fo = L.FitOut(*[_ptr(out[k]) for k in ("par_in", "par_out", "cov_out", "chi2", "n_hits",
                                             "n_members", "status")])
    cuts = merge_cuts(sectors_per_side)
    up, dn, grp = links
    L.check(L.lib().tpc_fit_merged_tracks(ctx.handle, C.byref(ev.problem), _clusters(ev),
                                          _tracklets(ev), _tracks(ev), status_count_ptr(ev),
                                          _ptr(up), _ptr(dn), _ptr(grp), int(sectors_per_side),
                                          cuts.cos_width, cuts.sin_width, int(n_pass),
                                          float(cov_scale), fo, _stream(stream)),
            "tpc_fit_merged_tracks")
    return out


def compress_clusters(ctx: Context, ev: Event, charge: torch.Tensor, qbits: int = 5,
                      cbits: int = 5, chunk: int = 4096, stream=None, state=None):
    """Cluster compression of a tracked event (section 6): returns (blob
    uint8 device tensor, its size as a device int64 tensor).  The blob buffer
    holds 16 bytes per cluster plus the tables; a larger blob (never seen on
    tracked events) raises.  `state` (a dict) keeps the buffers between
    calls."""
    dev = ev.t["row"].device
    state = {} if state is None else state
    need = C.c_size_t(0)
    L.check(L.lib().tpc_compress_workspace_size(C.byref(ev.problem), ev.track_capacity,
                                                ev.track_hit_capacity, int(chunk),
                                                C.byref(need)), "tpc_compress_workspace_size")
    if "ws" not in state or state["ws"].numel() < need.value:
        state["ws"] = torch.empty(max(need.value, 1), dtype=torch.uint8, device=dev)
    cap = 16 * int(ev.problem.n_clusters) + 16 * ev.track_capacity + (1 << 20)
    if "out" not in state or state["out"].numel() < cap:
        state["out"] = torch.empty(cap, dtype=torch.uint8, device=dev)
        state["size"] = torch.zeros(1, dtype=torch.int64, device=dev)
    cp = L.CompressParams(int(qbits), int(cbits), int(chunk))
    ch = charge.detach().to(device=dev, dtype=torch.float32).contiguous()
    state["charge"] = ch
    L.check(L.lib().tpc_compress_clusters(ctx.handle, C.byref(ev.problem), _clusters(ev),
                                          _ptr(ch), _grid(ev), _tracklets(ev), _tracks(ev),
                                          status_count_ptr(ev), cp, _ptr(state["out"]),
                                          state["out"].numel(), _ptr(state["size"]),
                                          _ptr(state["ws"]), state["ws"].numel(),
                                          _stream(stream)), "tpc_compress_clusters")
    return state["out"], state["size"]


def track_t0(ctx: Context, ev: Event, vd: float = 2.58, stream=None):
    """Interaction time of the event's found tracks in continuous read-out
    (after the tracking calls): device tensors (z0, y0, t0 float32, ok int8)
    of tracks.capacity entries; the first n_tracks of them are written."""
    dev = ev.t["row"].device
    cap = max(ev.track_capacity, 1)
    out = [torch.empty(cap, dtype=torch.float32, device=dev) for _ in range(3)]
    ok = torch.empty(cap, dtype=torch.int8, device=dev)
    L.check(L.lib().tpc_track_t0(ctx.handle, C.byref(ev.problem), _tracklets(ev), _tracks(ev),
                                 status_count_ptr(ev), float(vd), *[_ptr(o) for o in out],
                                 _ptr(ok), _stream(stream)),
            "tpc_track_t0")
    return out[0], out[1], out[2], ok


def get_status(ev: Event, stream=None) -> dict:
    st = L.Status()
    L.check(L.lib().tpc_get_status(_ptr(ev.t["ws"]), C.byref(st), _stream(stream)),
            "tpc_get_status")
    return {name: getattr(st, name) for name, _ in L.Status._fields_ if name != "pad_"}


def track(ctx: Context, ev: Event, stream=None):
    """The four tracking calls in order on one stream."""
    build_grid(ctx, ev, stream)
    find_neighbours(ctx, ev, stream)
    construct_tracklets(ctx, ev, stream)
    select_tracks(ctx, ev, stream)


def results(ev: Event, stream=None) -> dict:
    """Host copies of every output, sliced to the counts in the status
    block.  Links are returned in grid-position space as the library
    writes them, plus the grid permutation to map them to cluster ids."""
    torch.cuda.current_stream().synchronize() if stream is None else stream.synchronize()
    st = get_status(ev, stream)
    t = ev.t
    n = int(st["n_grid"])
    m = min(int(st["n_starts"]), ev.start_capacity)
    nt = min(int(st["n_tracks"]), ev.track_capacity)
    out = dict(status=st)
    cpu = lambda x: x.cpu().numpy()
    out["bin_start"] = cpu(t["bin_start"])
    for k in ("yg", "zg", "idg", "up0", "down0", "up", "down"):
        out[k] = cpu(t[k][:n])
    out["starts"] = cpu(t["starts"][:m])
    out["t_start"] = cpu(t["t_start"][:m])
    # [row][tracklet] on the device; [tracklet][row] here
    out["t_hits"] = np.ascontiguousarray(
        cpu(t["t_hits"]).reshape(ev.n_rows, ev.start_capacity)[:, :m].T)
    out["t_nhits"] = cpu(t["t_nhits"][:m])
    out["t_rin"] = cpu(t["t_rin"][:m])
    out["t_par"] = cpu(t["t_par"][:m * 5]).reshape(m, 5)
    out["t_cov"] = cpu(t["t_cov"][:m * 15]).reshape(m, 15)
    out["t_chi2"] = cpu(t["t_chi2"][:m])
    off = cpu(t["trk_off"][:nt + 1])
    out["trk_off"] = off
    out["trk_hits"] = cpu(t["trk_hits"][:int(off[-1]) if nt > 0 else 0])
    out["trk_tracklet"] = cpu(t["trk_tracklet"][:nt])
    out["trk_side"] = cpu(t["trk_side"][:nt])
    return out


def status_count_ptr(ev: Event, field_name: str = "n_tracks") -> C.c_void_p:
    """Device address of a counter of the workspace status block."""
    off = getattr(L.Status, field_name).offset
    return C.c_void_p(ev.t["ws"].data_ptr() + off)


def found_track_hits(ev: Event, copies: bool = False) -> "TrackHits":
    """The tracks of an event as refit input, without a host round trip:
    the CSR the selection wrote, the tracks' sides and the device track
    count of the status block.  copies=False: the hits are the event's
    clusters gathered through the track's cluster ids (hit gradients then
    belong to clusters); copies=True: the selection's track-ordered copies
    of the hits' rows and coordinates, read as contiguous runs (the same
    values; hit gradients per track entry)."""
    t = ev.t
    if copies:
        return TrackHits(off=t["trk_off"], row=t["trk_row"], y=t["trk_y"], z=t["trk_z"],
                         side=t["trk_side"], idx=None, d_count=status_count_ptr(ev),
                         n_tracks_cap=ev.track_capacity, n_hits_cap=ev.track_hit_capacity)
    return TrackHits(off=t["trk_off"], row=t["row"], y=t["y"], z=t["z"], side=t["trk_side"],
                     idx=t["trk_hits"], d_count=status_count_ptr(ev),
                     n_tracks_cap=ev.track_capacity, n_hits_cap=ev.track_hit_capacity)


def timing_enable(ctx: Context, on: bool = True):
    L.check(L.lib().tpc_timing_enable(ctx.handle, 1 if on else 0), "tpc_timing_enable")


def timing_report(ctx: Context, max_kernels: int = 64) -> dict:
    """{kernel name: (launches, total ms)} since the last report."""
    names = (C.c_char_p * max_kernels)()
    launches = (C.c_int64 * max_kernels)()
    ms = (C.c_double * max_kernels)()
    n = C.c_int()
    L.check(L.lib().tpc_timing_report(ctx.handle, max_kernels, names, launches, ms, C.byref(n)),
            "tpc_timing_report")
    return {names[i].decode(): (int(launches[i]), float(ms[i]))
            for i in range(min(n.value, max_kernels))}


# ---------------------------------------------------------------- refit

CALIB_MODEL = dict(drift_len=250.0, vd=2.58, tan_half=0.17632698070846498, u_centre=165.0,
                   u_scale=80.0)


def calib_struct(cm=None) -> L.CalibModel:
    cm = dict(CALIB_MODEL, **(cm or {}))
    return L.CalibModel(*(cm[k] for k, _ in L.CalibModel._fields_))


@dataclass
class TrackHits:
    """Refit input: CSR over tracks; entry j is cluster idx[j] of row/y/z
    (or cluster j without idx).  With d_count (device address of an int64
    count) the number of tracks is read on the device, up to n_tracks_cap."""
    off: torch.Tensor      # int32 [n_tracks + 1]
    row: torch.Tensor      # uint8 [n_clusters]
    y: torch.Tensor        # float32 [n_clusters]
    z: torch.Tensor        # float32 [n_clusters]
    side: torch.Tensor | None = None   # int8 [n_tracks]
    idx: torch.Tensor | None = None    # int32 [n_hits]
    d_count: C.c_void_p | None = None
    n_tracks_cap: int | None = None
    n_hits_cap: int | None = None

    @property
    def n_tracks(self):
        return int(self.n_tracks_cap if self.n_tracks_cap is not None else self.off.shape[0] - 1)

    @property
    def n_hits(self):
        if self.n_hits_cap is not None:
            return int(self.n_hits_cap)
        return int(self.idx.shape[0] if self.idx is not None else self.row.shape[0])

    def struct(self, y=None, z=None) -> L.TrackHits:
        return L.TrackHits(_ptr(self.off), _ptr(self.idx), _ptr(self.row),
                           _ptr(self.y if y is None else y), _ptr(self.z if z is None else z),
                           _ptr(self.side), self.d_count, self.n_tracks, self.n_hits)


def checkpoint_bytes(n_tracks: int, n_rows: int) -> int:
    """Size of the refit checkpoint buffer for n_tracks tracks of at most
    n_rows hits."""
    nb = C.c_size_t()
    L.check(L.lib().tpc_refit_checkpoint_size(int(n_tracks), int(n_rows), C.byref(nb)),
            "tpc_refit_checkpoint_size")
    return int(nb.value)


def _nbytes(t) -> int:
    return 0 if t is None else t.numel() * t.element_size()


def refit(ctx: Context, hits: TrackHits, row_x: torch.Tensor, prm: dict, theta: torch.Tensor,
          checkpoints: bool = True, cm=None, stream=None, y=None, z=None, out=None):
    """Forward refit; returns dict(par, cov, chi2, status, checkpoints).
    `out` (a dict returned by an earlier call of the same size) is reused."""
    dev = hits.row.device
    n = hits.n_tracks
    if out is None:
        out = dict(par=torch.empty(n * 5, dtype=torch.float32, device=dev),
                   cov=torch.empty(n * 15, dtype=torch.float32, device=dev),
                   chi2=torch.empty(n, dtype=torch.float32, device=dev),
                   status=torch.empty(n, dtype=torch.int32, device=dev))
        out["checkpoints"] = (torch.empty(max(checkpoint_bytes(n, int(row_x.shape[0])) // 4, 1),
                                          dtype=torch.float32, device=dev)
                              if checkpoints else None)
    else:
        out = dict(out)
    P = params_struct(prm)
    CM = calib_struct(cm)
    th = theta.detach().to(device=dev, dtype=torch.float32).contiguous()
    L.check(L.lib().tpc_refit(ctx.handle, hits.struct(y, z), int(row_x.shape[0]), _ptr(row_x),
                              C.byref(P), C.byref(CM), _ptr(th), _ptr(out["par"]),
                              _ptr(out["cov"]), _ptr(out["chi2"]), _ptr(out["status"]),
                              _ptr(out["checkpoints"]), _nbytes(out["checkpoints"]),
                              _stream(stream)), "tpc_refit")
    out["par"] = out["par"].view(n, 5)
    out["cov"] = out["cov"].view(n, 15)
    return out


def refit_adjoint(ctx: Context, hits: TrackHits, row_x: torch.Tensor, prm: dict,
                  theta: torch.Tensor, fwd: dict, grad_chi2: torch.Tensor, cm=None, stream=None,
                  y=None, z=None, out=None, grad_par=None, grad_x=None):
    """Gradients of sum_k grad_chi2[k] chi2[k] (+ sum_k grad_par[k] . par[k]
    + sum_k grad_x[k] x_last[k] when either seed is given): (grad_y, grad_z,
    grad_theta), grad_y/grad_z per hit entry of the track list.  `out` (dict
    with ws, gy, gz, gt of an earlier call, or any of them) is reused;
    entries of tracks past the device track count are not written."""
    dev = hits.row.device
    nb = C.c_size_t()
    L.check(L.lib().tpc_refit_workspace_size(hits.n_tracks, C.byref(nb)), "workspace")
    out = {} if out is None else out
    if "ws" not in out:
        out["ws"] = torch.empty(max(int(nb.value), 64), dtype=torch.uint8, device=dev)
    if "gy" not in out:
        out["gy"] = torch.empty(max(hits.n_hits, 1), dtype=torch.float32, device=dev)
        out["gz"] = torch.empty(max(hits.n_hits, 1), dtype=torch.float32, device=dev)
    if "gt" not in out:
        out["gt"] = torch.zeros(16, dtype=torch.float32, device=dev)
    ws, gy, gz, gt = out["ws"], out["gy"], out["gz"], out["gt"]
    P = params_struct(prm)
    CM = calib_struct(cm)
    th = theta.detach().to(device=dev, dtype=torch.float32).contiguous()
    g = grad_chi2.detach().to(device=dev, dtype=torch.float32).contiguous()
    if grad_par is None and grad_x is None:
        L.check(L.lib().tpc_refit_adjoint(ctx.handle, hits.struct(y, z), int(row_x.shape[0]),
                                          _ptr(row_x), C.byref(P), C.byref(CM), _ptr(th),
                                          _ptr(fwd["checkpoints"]), _nbytes(fwd["checkpoints"]),
                                          _ptr(fwd["status"]), _ptr(g),
                                          _ptr(gy), _ptr(gz), _ptr(gt), _ptr(ws), int(nb.value),
                                          _stream(stream)), "tpc_refit_adjoint")
    else:
        L.check(L.lib().tpc_refit_adjoint_seeded(
            ctx.handle, hits.struct(y, z), int(row_x.shape[0]), _ptr(row_x), C.byref(P),
            C.byref(CM), _ptr(th), _ptr(fwd["checkpoints"]), _nbytes(fwd["checkpoints"]),
            _ptr(fwd["status"]), _ptr(g), _ptr(grad_par), _ptr(grad_x), _ptr(gy), _ptr(gz),
            _ptr(gt), _ptr(ws), int(nb.value), _stream(stream)), "tpc_refit_adjoint_seeded")
    return gy[:hits.n_hits], gz[:hits.n_hits], gt


def vertex_residual(ctx: Context, hits: TrackHits, row_x: torch.Tensor, prm: dict,
                    theta: torch.Tensor, fwd: dict, sigma_v: float = 0.01, weights=None, cm=None,
                    stream=None, out=None):
    """Beam-axis term of the calibration objective for every track of the
    refit `fwd` (with its covariance): (loss [n], grad_par [n, 5], grad_x [n],
    ok [n], weights [n, 3]) device tensors.  weights: held per-track weights
    (an earlier call's), or None to take them from the refit covariance.
    `out` (the dict of an earlier call of the same size) is reused."""
    dev = hits.row.device
    n = max(hits.n_tracks, 1)
    out = {} if out is None else out
    if "loss" not in out:
        out["loss"] = torch.empty(n, dtype=torch.float32, device=dev)
        out["gp"] = torch.empty(n, 5, dtype=torch.float32, device=dev)
        out["gx"] = torch.empty(n, dtype=torch.float32, device=dev)
        out["ok"] = torch.empty(n, dtype=torch.int8, device=dev)
        out["w"] = torch.empty(n, 3, dtype=torch.float32, device=dev)
    P = params_struct(prm)
    CM = calib_struct(cm)
    th = theta.detach().to(device=dev, dtype=torch.float32).contiguous()
    L.check(L.lib().tpc_vertex_residual(ctx.handle, hits.struct(), int(row_x.shape[0]),
                                        _ptr(row_x), C.byref(P), C.byref(CM), _ptr(th),
                                        _ptr(fwd["par"]), _ptr(fwd["cov"]), _ptr(fwd["status"]),
                                        float(sigma_v), _ptr(weights),
                                        _ptr(out["w"]) if weights is None else None,
                                        _ptr(out["loss"]), _ptr(out["gp"]), _ptr(out["gx"]),
                                        _ptr(out["ok"]), _stream(stream)),
            "tpc_vertex_residual")
    return out["loss"], out["gp"], out["gx"], out["ok"], (out["w"] if weights is None
                                                          else weights)


# parameters the calibration fits by default: t0 and the azimuthal distortion
# terms that move clusters without rescaling the measured coordinates
# (functions of the row and the drift only: 1, u, u^2, w).  The drift velocity
# scale is not separable from t0 for primaries of a known vertex on one z
# side; the radial terms move the row planes along the track, which the track
# curvature nearly absorbs (the chi2 pins them only weakly and with a bias of
# many statistical errors); the terms in the raw y rescale the cluster
# errors, which a chi2 objective rewards (it prefers shrunken coordinates):
# those stay at theta0.
CALIB_FREE = (1, 9, 10, 12, 15)


def calibration_objective(ctx: Context, hits: TrackHits, row_x: torch.Tensor, prm: dict,
                          theta: torch.Tensor, weights=None, sigma_v: float = 0.01, cm=None,
                          stream=None, state=None, grad=True):
    """Calibration objective with the beam-axis constraint (section 3,
    online calibration; section 2, primaries from the origin):
    L(theta) = sum_k chi2_k(theta) + r_k^T W_k r_k over the tracks of `hits`,
    r_k the refit state of the last hit at the beam-axis plane, W_k held
    weights (None: taken from this refit's covariance), computed by the
    refit, the beam-axis kernel and the seeded adjoint.  Returns (L as a
    float, dL/dtheta float32 [16] device tensor or None, the weights).
    `state` (a dict) keeps the buffers between calls."""
    state = {} if state is None else state
    state["fwd"] = refit(ctx, hits, row_x, prm, theta, cm=cm, stream=stream,
                         out=state.get("fwd"))
    fwd = state["fwd"]
    state.setdefault("vtx", {})
    loss, gp, gx, ok, w = vertex_residual(ctx, hits, row_x, prm, theta, fwd, sigma_v, weights,
                                          cm, stream, out=state["vtx"])
    n = hits.n_tracks
    val = float(fwd["chi2"][:n].double().sum() + loss[:n].double().sum())
    if not grad:
        return val, None, w
    if "g1" not in state:
        state["g1"] = torch.ones(max(n, 1), dtype=torch.float32, device=hits.row.device)
    state.setdefault("adj", {})
    _, _, gt = refit_adjoint(ctx, hits, row_x, prm, theta, fwd, state["g1"], cm=cm,
                             stream=stream, out=state["adj"], grad_par=gp, grad_x=gx)
    return val, gt, w


def calibrate(ctx: Context, hits: TrackHits, row_x: torch.Tensor, prm: dict, theta0,
              free=CALIB_FREE, sigma_v: float = 0.01, n_iter: int = 12, fd_step: float = 1e-4,
              cm=None, stream=None):
    """Global calibration (section 3's online calibration) by damped Newton
    (Levenberg-Marquardt) steps on the calibration objective: each iteration
    takes the beam-axis weights at the current theta and holds them, the
    gradient is the adjoint's, the Hessian over the free parameters is taken
    by central differences of that gradient (step fd_step), and a step is
    kept only when the objective decreases (else the damping grows).  free:
    the indices of theta to fit; the others stay at theta0.  Returns dict
    theta (float64 numpy [16]), objective, history, hessian (free x free),
    cov = 2 H^-1 and sigma (the estimator's statistical errors)."""
    import numpy as np
    free = np.asarray(free)
    th = np.asarray(theta0, np.float64).copy()
    dev = hits.row.device
    state = {}

    def f(t, w, grad=True):
        v, g, w2 = calibration_objective(ctx, hits, row_x, prm, torch.as_tensor(t, device=dev),
                                         w, sigma_v, cm, stream, state, grad)
        return v, (g.double().cpu().numpy() if g is not None else None), w2

    hist = []
    lam = 1e-3
    H = None
    for it in range(n_iter):
        val, g, w = f(th, None)
        w = w.clone()
        H = np.zeros((free.size, free.size))
        for j, k in enumerate(free):
            e = np.zeros(16)
            e[k] = fd_step
            H[:, j] = (f(th + e, w)[1][free] - f(th - e, w)[1][free]) / (2.0 * fd_step)
        H = 0.5 * (H + H.T)
        D = np.diag(np.diag(H))
        moved = False
        while lam < 1e12:
            step = -np.linalg.solve(H + lam * D, g[free])
            cand = th.copy()
            cand[free] += step
            v_new = f(cand, w, grad=False)[0]
            if v_new < val:
                th = cand
                lam = max(lam / 3.0, 1e-9)
                moved = True
                break
            lam *= 10.0
        hist.append(dict(objective=val, step=float(np.abs(step).max()) if moved else 0.0,
                         damping=lam))
        if not moved:
            break
    cov = 2.0 * np.linalg.inv(H)
    val = f(th, None, grad=False)[0]
    return dict(theta=th, objective=val, history=hist, free=free, hessian=H, cov=cov,
                sigma=np.sqrt(np.abs(np.diag(cov))))

"""ctypes declarations of the C ABI in include/tpc.h (argument marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
SO = os.path.join(HERE, "libtpc.so")

P = C.c_void_p
I32 = C.c_int32
I64 = C.c_int64
F32 = C.c_float


class Params(C.Structure):
    _fields_ = [(n, F32) for n in (
        "curv", "nb_win_y", "nb_win_z", "nb_d2max", "sigma_y2", "sigma_z2", "chi2_max",
        "search_nsigma", "s_max", "c_ss0", "c_tt0", "c_ww0")] + \
        [(n, I32) for n in ("max_miss", "min_tracklet_hits", "min_track_hits")]


class Problem(C.Structure):
    _fields_ = [("n_sectors", I32), ("n_rows", I32), ("n_clusters", I64), ("n_bins", I64),
                ("h_sectors", P), ("d_sectors", P), ("d_row_x", P), ("params", Params)]


class Clusters(C.Structure):
    _fields_ = [("row", P), ("y", P), ("z", P)]


class Grid(C.Structure):
    _fields_ = [("bin_start", P), ("y", P), ("z", P), ("id", P)]


class Links(C.Structure):
    _fields_ = [("up0", P), ("down0", P), ("up", P), ("down", P)]


class Starts(C.Structure):
    _fields_ = [("pos", P), ("capacity", I64)]


class Tracklets(C.Structure):
    _fields_ = [("start", P), ("hits", P), ("nhits", P), ("row_inner", P), ("par", P),
                ("cov", P), ("chi2", P), ("capacity", I64)]


class Tracks(C.Structure):
    _fields_ = [("off", P), ("hits", P), ("tracklet", P), ("side", P), ("capacity", I64),
                ("hit_capacity", I64), ("hit_row", P), ("hit_y", P), ("hit_z", P)]


class Status(C.Structure):
    _fields_ = [("n_grid", I64), ("n_bad_rows", I64), ("n_starts", I64), ("n_tracks", I64),
                ("n_track_hits", I64), ("overflow", I32), ("pad_", I32),
                ("n_propagations", I64), ("n_updates", I64), ("n_candidates", I64)]


class CalibModel(C.Structure):
    _fields_ = [(n, F32) for n in ("drift_len", "vd", "tan_half", "u_centre", "u_scale")]


class MergeCuts(C.Structure):
    _fields_ = [("sectors_per_side", C.c_int32), ("cos_width", C.c_float),
                ("sin_width", C.c_float), ("inv_window", C.c_float * 5)]


class CompressParams(C.Structure):
    _fields_ = [("qbits", C.c_int32), ("cbits", C.c_int32), ("chunk", C.c_int32)]


class FitOut(C.Structure):
    _fields_ = [("par_in", P), ("par_out", P), ("cov_out", P), ("chi2", P), ("n_hits", P),
                ("n_members", P), ("status", P)]


class Tuning(C.Structure):
    _fields_ = [("tracklet_form", C.c_int32), ("neighbour_block", C.c_int32),
                ("persistent_scale", C.c_int32), ("persistent_blocks_per_cu", C.c_int32)]


class TrackHits(C.Structure):
    _fields_ = [("off", P), ("idx", P), ("row", P), ("y", P), ("z", P), ("side", P),
                ("d_count", P), ("n_tracks", I64), ("n_hits", I64)]


EXPORTS = {
    "tpc_context_create": (C.c_int, [C.POINTER(P), C.c_int]),
    "tpc_context_destroy": (C.c_int, [P]),
    "tpc_context_set_tuning": (C.c_int, [P, C.POINTER(Tuning)]),
    "tpc_context_get_tuning": (C.c_int, [P, C.POINTER(Tuning)]),
    "tpc_workspace_size": (C.c_int, [C.POINTER(Problem), I64, C.POINTER(C.c_size_t)]),
    "tpc_build_grid": (C.c_int, [P, C.POINTER(Problem), Clusters, Grid, P, C.c_size_t, P]),
    "tpc_find_neighbours": (C.c_int, [P, C.POINTER(Problem), Grid, Links, Starts, P,
                                      C.c_size_t, P]),
    "tpc_construct_tracklets": (C.c_int, [P, C.POINTER(Problem), Grid, Links, Starts,
                                          Tracklets, P, C.c_size_t, P]),
    "tpc_select_tracks": (C.c_int, [P, C.POINTER(Problem), Grid, Tracklets, Tracks, P,
                                    C.c_size_t, P]),
    "tpc_get_status": (C.c_int, [P, C.POINTER(Status), P]),
    "tpc_track_batch": (C.c_int, [P, C.POINTER(Problem), Clusters, Grid, Links, Starts,
                                  Tracklets, Tracks, P, C.c_size_t, C.c_int, C.c_int, P]),
    "tpc_refit": (C.c_int, [P, TrackHits, I32, P, C.POINTER(Params), C.POINTER(CalibModel), P,
                            P, P, P, P, P, C.c_size_t, P]),
    "tpc_refit_checkpoint_size": (C.c_int, [I64, I32, C.POINTER(C.c_size_t)]),
    "tpc_refit_workspace_size": (C.c_int, [I64, C.POINTER(C.c_size_t)]),
    "tpc_refit_adjoint": (C.c_int, [P, TrackHits, I32, P, C.POINTER(Params),
                                    C.POINTER(CalibModel), P, P, C.c_size_t, P, P, P, P, P, P,
                                    C.c_size_t, P]),
    "tpc_refit_adjoint_seeded": (C.c_int, [P, TrackHits, I32, P, C.POINTER(Params),
                                           C.POINTER(CalibModel), P, P, C.c_size_t, P, P, P, P,
                                           P, P, P, P, C.c_size_t, P]),
    "tpc_vertex_residual": (C.c_int, [P, TrackHits, I32, P, C.POINTER(Params),
                                      C.POINTER(CalibModel), P, P, P, P, F32, P, P, P, P, P, P,
                                      P]),
    "tpc_refit_adjoint_noalloc": (C.c_int, [P, TrackHits, I32, P, C.POINTER(Params),
                                            C.POINTER(CalibModel), P, P, C.c_size_t, P, P, P,
                                            P, P, P]),
    "tpc_attach_workspace_size": (C.c_int, [C.POINTER(Problem), C.POINTER(C.c_size_t)]),
    "tpc_attach_clusters": (C.c_int, [P, C.POINTER(Problem), Clusters, Grid, Tracklets, Tracks,
                                      P, F32, F32, P, P, P, C.c_size_t, P]),
    "tpc_merge_workspace_size": (C.c_int, [C.POINTER(Problem), I64, C.POINTER(C.c_size_t)]),
    "tpc_merge_sector_tracks": (C.c_int, [P, C.POINTER(Problem), Tracklets, Tracks, P, MergeCuts,
                                          P, P, P, P, C.c_size_t, P]),
    "tpc_compress_workspace_size": (C.c_int, [C.POINTER(Problem), I64, I64, I32,
                                              C.POINTER(C.c_size_t)]),
    "tpc_compress_clusters": (C.c_int, [P, C.POINTER(Problem), Clusters, P, Grid, Tracklets,
                                        Tracks, P, CompressParams, P, I64, P, P, C.c_size_t, P]),
    "tpc_fit_merged_tracks": (C.c_int, [P, C.POINTER(Problem), Clusters, Tracklets, Tracks, P,
                                        P, P, P, I32, F32, F32, I32, F32, FitOut, P]),
    "tpc_track_t0": (C.c_int, [P, C.POINTER(Problem), Tracklets, Tracks, P, F32, P, P, P, P, P]),
    "tpc_status_string": (C.c_char_p, [C.c_int]),
    "tpc_timing_enable": (C.c_int, [P, C.c_int]),
    "tpc_timing_report": (C.c_int, [P, C.c_int, C.POINTER(C.c_char_p), C.POINTER(I64),
                                    C.POINTER(C.c_double), C.POINTER(C.c_int)]),
}

_lib = None


def lib():
    """The loaded libtpc.so.  Raises if it has not been built: there is no
    fallback implementation."""
    global _lib
    if _lib is None:
        if not os.path.exists(SO):
            raise ImportError(f"{SO} is missing: build it with "
                              "`python -m paper_1905_05515_amd.build` (hipcc, gfx950)")
        L = C.CDLL(SO)
        for name, (res, args) in EXPORTS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


class TPCError(RuntimeError):
    pass


def check(code: int, what: str):
    if code != 0:
        msg = lib().tpc_status_string(code).decode()
        raise TPCError(f"{what}: {msg} (code {code})")

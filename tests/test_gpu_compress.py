"""Cluster compression on the GPU (tpc_compress_clusters) against the
oracle, byte for byte: the blob of a tracked event (the oracle's from its
own tracking of the same event) on the single sector, the central event and
a three-collision continuous read-out slice, and with other precisions and
chunk sizes; the oracle decodes the GPU's blob to the quantised clusters."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_common import ctx, run_gpu, run_oracle
from paper_1905_05515_amd import _lib as L
from paper_1905_05515_amd import api

pytestmark = pytest.mark.gpu
PRM = synth.default_params()


def _check(ev, qbits=5, cbits=5, chunk=4096):
    e, g = run_gpu(ev)
    blob, size = api.compress_clusters(ctx(), e, torch.as_tensor(ev.charge), qbits, cbits, chunk)
    torch.cuda.synchronize()
    n = int(size.item())
    gb = blob[:n].cpu().numpy()
    o = run_oracle(ev, layout=e.layout)
    trk, trl = o["tracks"], o["tracklets"]
    tt = trk["trk_tracklet"]
    tab, _ = e.layout
    ob = oracle.compress(tab, 152, ev.row_x, PRM, ev.row, ev.y, ev.z, ev.charge, o["grid"],
                         trk["trk_off"], trk["trk_hits"], trl["par"][tt], trl["row_inner"][tt],
                         qbits=qbits, cbits=cbits, chunk=chunk)
    assert n == ob.size, (n, ob.size)
    assert np.array_equal(gb, ob)
    return gb


@pytest.mark.timeout(600)
def test_compression_matches_the_oracle_byte_for_byte():
    ev = synth.make_config1()
    print(f"case compress c1 n={ev.n_clusters}", flush=True)
    _check(ev)
    _check(ev, qbits=3, cbits=4, chunk=64)
    _check(ev, chunk=1000)             # chunks that do not start on 16-byte boundaries
    ev = synth.make_config2()
    print(f"case compress c2 n={ev.n_clusters}", flush=True)
    _check(ev, chunk=16384)
    blob = _check(ev)
    d = oracle.decompress(blob, ev.n_clusters, ev.row_x, PRM)
    assert d["row"].size == ev.n_clusters
    assert blob.size < 3.0 * ev.n_clusters


@pytest.mark.timeout(600)
def test_compression_continuous_slice():
    ev = synth.make_config3(n_collisions=3)
    print(f"case compress c3 3 collisions n={ev.n_clusters}", flush=True)
    _check(ev, chunk=4096)


def test_compression_small_output_and_bad_arguments():
    ev = synth.make_config1()
    print("case compress bad arguments", flush=True)
    e, g = run_gpu(ev)
    ch = torch.as_tensor(ev.charge)
    for kw in (dict(qbits=13), dict(cbits=1), dict(chunk=16)):
        with pytest.raises(L.TPCError):
            api.compress_clusters(ctx(), e, ch, **kw)
    # too small an output: the size is reported, nothing written
    state = {"out": torch.zeros(64, dtype=torch.uint8, device="cuda"),
             "size": torch.zeros(1, dtype=torch.int64, device="cuda")}
    import ctypes as C
    need = C.c_size_t(0)
    L.lib().tpc_compress_workspace_size(C.byref(e.problem), e.track_capacity,
                                        e.track_hit_capacity, 16384, C.byref(need))
    ws = torch.empty(need.value, dtype=torch.uint8, device="cuda")
    chd = ch.cuda()
    rc = L.lib().tpc_compress_clusters(ctx().handle, C.byref(e.problem), api._clusters(e),
                                       api._ptr(chd), api._grid(e), api._tracklets(e),
                                       api._tracks(e), api.status_count_ptr(e),
                                       L.CompressParams(5, 5, 16384), api._ptr(state["out"]), 64,
                                       api._ptr(state["size"]), api._ptr(ws), ws.numel(), None)
    assert rc == 0
    torch.cuda.synchronize()
    assert int(state["size"].item()) > 64
    assert int(state["out"].sum().item()) == 0


def test_compression_with_and_without_the_hit_copies():
    """The tracks' hit copies are read in place of the gathered cluster
    values: without them the blob is the same; one or two of them null is an
    argument error."""
    import ctypes as C
    ev = synth.make_config1()
    print("case compress hit copies c1", flush=True)
    e, g = run_gpu(ev)
    ch = torch.as_tensor(ev.charge)
    blob, size = api.compress_clusters(ctx(), e, ch)
    torch.cuda.synchronize()
    ref = blob[:int(size.item())].cpu().numpy().copy()
    need = C.c_size_t(0)
    L.lib().tpc_compress_workspace_size(C.byref(e.problem), e.track_capacity,
                                        e.track_hit_capacity, 4096, C.byref(need))
    ws = torch.empty(need.value, dtype=torch.uint8, device="cuda")
    out = torch.zeros(ref.size + 4096, dtype=torch.uint8, device="cuda")
    sz = torch.zeros(1, dtype=torch.int64, device="cuda")
    chd = ch.cuda()

    def call(trk):
        return L.lib().tpc_compress_clusters(ctx().handle, C.byref(e.problem), api._clusters(e),
                                             api._ptr(chd), api._grid(e), api._tracklets(e), trk,
                                             api.status_count_ptr(e), L.CompressParams(5, 5, 4096),
                                             api._ptr(out), out.numel(), api._ptr(sz),
                                             api._ptr(ws), ws.numel(), None)

    trk = api._tracks(e)
    trk.hit_row = trk.hit_y = trk.hit_z = None
    assert call(trk) == 0
    torch.cuda.synchronize()
    assert int(sz.item()) == ref.size
    assert np.array_equal(out[:ref.size].cpu().numpy(), ref)
    trk = api._tracks(e)
    trk.hit_z = None
    assert call(trk) == 1            # TPC_ERR_INVALID_ARG

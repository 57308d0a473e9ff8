"""Pins of the oracle's cluster compression (section 6, steps 2 to 4:
integer cluster format with the resolution's precision and a charge
precision relative to its value, residuals to tracks for clusters on tracks
and position differences otherwise, entropy coding; rANS is one of the
coders the paper names).

  * rANS: every byte stream comes back bit for bit (uniform, skewed, single
    symbol, every symbol once), and its size is the Shannon entropy of the
    stream under the coder's own 12-bit table plus at most 0.1% and the
    4-byte final state;
  * charge: codes decode within a relative 2^-5 of the count (exact below
    2^5), are monotonic and fit a byte;
  * whole events (a single sector and the central event): decompression
    returns every cluster's row, y and z in units of 2^-5 cm (within half a
    unit of the float value) and charge code, clusters on tracks track by
    track, the others in grid order;
  * a truncated or corrupted blob is refused.
"""
import numpy as np
import pytest

import oracle
import synth
from paper_1905_05515_amd.layout import grid_layout

PRM = synth.default_params()


def _table_entropy_bits(sym):
    """Bits of the stream under the coder's normalised 12-bit frequencies
    (the normalisation written out again in numpy)."""
    cnt = np.bincount(sym, minlength=256).astype(np.int64)
    total = cnt.sum()
    f = np.where(cnt > 0, np.maximum(cnt * 4096 // total, 1), 0)
    while f.sum() > 4096:
        i = int(np.argmax(np.where(f > 1, f, -1)))
        f[i] -= 1
    while f.sum() < 4096:
        i = int(np.argmax(np.where(cnt > 0, cnt, -1)))
        f[i] += 1
    return float(np.sum(cnt[cnt > 0] * -np.log2(f[cnt > 0] / 4096.0)))


@pytest.mark.parametrize("kind", ["uniform", "geometric", "single", "all"])
def test_rans_roundtrip_and_size(kind):
    rng = np.random.default_rng(4)
    n = 200_000
    if kind == "uniform":
        sym = rng.integers(0, 256, n)
    elif kind == "geometric":
        sym = np.minimum(rng.geometric(0.3, n) - 1, 255)
    elif kind == "single":
        sym = np.full(n, 7)
    else:
        sym = np.arange(256).repeat(3)
        rng.shuffle(sym)
    sym = sym.astype(np.uint8)
    by, back = oracle.rans_roundtrip(sym)
    assert np.array_equal(back, sym)
    bits = _table_entropy_bits(sym)
    assert by.size * 8 <= bits * 1.001 + 32 + 8, (by.size * 8, bits)
    assert by.size * 8 >= bits - 8


def test_charge_codes():
    def code(x):
        # the definition written out again: below 2^5 exact, above it the
        # exponent and the four bits after the leading one
        if x < 32:
            return x
        e = int(x).bit_length() - 5
        return 32 + (e - 1) * 16 + ((x >> e) - 16)
    vv = np.arange(0, 65536, 7)
    dec = np.array([oracle.charge_decode(code(int(x))) for x in vv])
    assert np.all(dec[vv < 32] == vv[vv < 32])
    big = vv >= 32
    assert np.all(np.abs(dec[big] - vv[big]) <= vv[big] / 32.0)
    cs = np.array([code(int(x)) for x in vv])
    assert np.all(np.diff(cs) >= 0) and cs.max() < 255


def _event_blob(ev):
    tab, nb = grid_layout(ev.sector_offsets, ev.sector_range, occupancy=0.125,
                          sides=ev.sector_side)
    o = oracle.track_event(ev.row, ev.y, ev.z, tab, nb, ev.row_x, PRM)
    trk, trl = o["tracks"], o["tracklets"]
    tt = trk["trk_tracklet"]
    blob = oracle.compress(tab, 152, ev.row_x, PRM, ev.row, ev.y, ev.z, ev.charge, o["grid"],
                           trk["trk_off"], trk["trk_hits"], trl["par"][tt],
                           trl["row_inner"][tt])
    return blob, o


def _check_roundtrip(ev):
    blob, o = _event_blob(ev)
    d = oracle.decompress(blob, ev.n_clusters, ev.row_x, PRM)
    trk = o["tracks"]
    off, hits = trk["trk_off"], trk["trk_hits"]
    na = int(off[-1])
    on = np.zeros(ev.n_clusters, bool)
    on[hits] = True
    idg = o["grid"]["idg"]
    order = np.concatenate([hits, idg[~on[idg]]])
    yq = np.rint(ev.y[order] * np.float32(32.0)).astype(np.int32)
    zq = np.rint(ev.z[order] * np.float32(32.0)).astype(np.int32)
    assert np.array_equal(d["row"], ev.row[order])
    assert np.array_equal(d["yq"], yq) and np.array_equal(d["zq"], zq)
    assert np.all(np.abs(d["yq"] / 32.0 - ev.y[order]) <= 1 / 64.0 + 1e-6)
    assert np.array_equal(d["track"][:na], np.repeat(np.arange(len(off) - 1), np.diff(off)))
    assert np.all(d["track"][na:] == -1)
    sec = np.searchsorted(ev.sector_offsets, order[na:], side="right") - 1
    assert np.array_equal(d["sector"][na:], sec)
    q = np.array([oracle.charge_decode(c) for c in d["qcode"][:2000]])
    ch = np.rint(ev.charge[order[:2000]])
    assert np.all(np.abs(q - ch) <= np.maximum(ch / 32.0, 0.0))
    return blob, d


def test_single_sector_roundtrip():
    _check_roundtrip(synth.make_config1())


def test_central_event_roundtrip_and_size():
    ev = synth.make_config2()
    blob, _ = _check_roundtrip(ev)
    # residuals to tracks keep the clusters on tracks far below the float
    # format's 13 bytes
    assert blob.size < 3.0 * ev.n_clusters


def test_malformed_blobs_are_refused():
    ev = synth.make_config1()
    blob, _ = _event_blob(ev)
    with pytest.raises(ValueError):
        oracle.decompress(blob[: blob.size // 2], ev.n_clusters, ev.row_x, PRM)
    bad = blob.copy()
    bad[0] ^= 1
    with pytest.raises(ValueError):
        oracle.decompress(bad, ev.n_clusters, ev.row_x, PRM)
    with pytest.raises(ValueError):
        oracle.decompress(blob, ev.n_clusters - 1, ev.row_x, PRM)

"""Host-side choice of the per-sector bin grid.

The grid only accelerates the searches: every decision of the tracker is an
exact predicate on cluster coordinates with ties broken on cluster ids, so
the tracks do not depend on the bin layout chosen here (the grid permutation
itself does).  The layout is a plain table that the caller hands to the
library together with the clusters.
"""
from __future__ import annotations

import math

import numpy as np

# one record per sector, mirrored by tpc_sector in include/tpc.h
SECTOR_DTYPE = np.dtype([
    ("y0", np.float32), ("z0", np.float32),
    ("inv_by", np.float32), ("inv_bz", np.float32),
    ("nby", np.int32), ("nbz", np.int32),
    ("bin_base", np.int32), ("side", np.int32),
    ("begin", np.int64), ("end", np.int64),
])


def grid_layout(sector_offsets, sector_range, n_rows=152, occupancy=2.0,
                max_bins_per_row=1 << 16, sides=None):
    """Bins per row chosen for about `occupancy` clusters per bin, split
    between y and z in proportion to the sector's extent; each sector has one
    more bin, after its rows, for clusters with an invalid row.

    sector_offsets: int [n_sectors + 1] cluster CSR; sector_range: float
    [n_sectors, 4] = (ymin, ymax, zmin, zmax); sides: +1/-1 per sector, by
    default -1 where the z range lies at or below 0.  Returns (table,
    n_bins) with table a SECTOR_DTYPE record array."""
    offs = np.asarray(sector_offsets, np.int64)
    rng = np.asarray(sector_range, np.float64)
    n_sec = offs.shape[0] - 1
    tab = np.zeros(n_sec, SECTOR_DTYPE)
    base = 0
    for s in range(n_sec):
        n = int(offs[s + 1] - offs[s])
        ylo, yhi, zlo, zhi = (float(v) for v in rng[s])
        ly = max(yhi - ylo, 1e-3)
        lz = max(zhi - zlo, 1e-3)
        nb = max(1.0, min(n / (n_rows * occupancy), float(max_bins_per_row)))
        nby = max(1, int(round(math.sqrt(nb * ly / lz))))
        nbz = max(1, int(round(nb / nby)))
        side = int(sides[s]) if sides is not None else (-1 if zhi <= 0.0 else 1)
        tab[s] = (np.float32(ylo), np.float32(zlo), np.float32(nby / ly),
                  np.float32(nbz / lz), nby, nbz, base, side, offs[s], offs[s + 1])
        base += n_rows * nby * nbz + 1      # + the bin of invalid rows
    if base >= 2**31 - 1:
        raise ValueError("bin grid too large for 32-bit bin indices")
    return tab, base

"""Seeded synthetic TPC workloads.

This package only produces inputs: helix tracks from a uniform 0.5 T field
crossing the pad-row planes of one or more TPC sectors, smeared, with noise,
optionally pile-up and calibration distortions.  It contains none of the
track-finding or fitting arithmetic; both the oracle and the HIP library
consume its arrays unchanged.
"""
from .events import (  # noqa: F401
    N_ROWS, ROW_X, CURV_PER_QPT, SIGMA, DRIFT_LEN, VD_CM_PER_US, TAN10,
    Event, RefitSet, make_event, make_sector_instance, make_config1,
    make_config2, make_config3, make_config4, make_config5, CONFIG_SEEDS,
    default_params, helix_plane_point,
)

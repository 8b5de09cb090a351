"""MI355X (gfx950) library for light-nucleus two-point correlators by Wick
contraction with baryon blocks (arXiv 2411.08962).

The C ABI is in ``include/wick.h``; :mod:`.wick` is its Python binding.
"""
from .wick import (BLOCK_LEN, ECORRUPT, EHIP, EINVAL, ENOMEM, EUNSUPPORTED, ETOOBIG, EXPORTS, OK,  # noqa: F401
                   PRECISIONS, GevpPlan, Plan, PointPlan, WickError, autotune, autotune_batch, blocks,
                   contract, contract_noalloc, correlator, gevp_contract, gevp_plan, gevp_plan_std, lib, plan, plan_std, plan_std_pair, point_blocks_correlator, point_correlator,
                   point_plan, point_plan_std,
                   profile, profile_read, version)

"""MI355X-native sparse wide/tall products y = A x and u^T = v^T A.

The work of one product is split among GPU workgroups by equal runs of
nonzeros (Eckstein & Matyasfalvi, arXiv:1812.00904, Section II); see
include/spw.h for the C ABI and ``spw`` for the Python binding.
"""
from .spw import (SPW_CSC, SPW_CSR, SPW_F64, SPW_F32, SPW_BF16, SPW_OP_MV, SPW_OP_VTM, SPW_PART_NONZERO,
                  SPW_PART_COLUMN, SPW_PART_MERGE, SPW_PLAN_AUTO, SPW_PLAN_SINGLE, SPW_PLAN_PASSES, SPW_PLAN_TILE, PLAN_NAMES,
                  Server, SpwError, spw_batch_plan, spw_set_batch_plan, spw_tune_cache_path,
                  SpwMatrix, create_opts, load,
                  spw_create, spw_create_coo, spw_destroy, spw_info, spw_mv, spw_vtm, spw_mv_batch, spw_vtm_batch, spw_cgls,
                  spw_plan_zones, spw_round_values, spw_profile_enable, spw_profile_select,
                  spw_profile_reset, spw_profile_read)

__all__ = ["SPW_CSC", "SPW_CSR", "SPW_F64", "SPW_F32", "SPW_BF16", "SPW_OP_MV", "SPW_OP_VTM", "SPW_PART_NONZERO",
           "SPW_PART_COLUMN", "SPW_PART_MERGE", "SPW_PLAN_AUTO", "SPW_PLAN_SINGLE", "SPW_PLAN_PASSES", "SPW_PLAN_TILE",
           "PLAN_NAMES", "Server", "spw_batch_plan", "spw_set_batch_plan", "spw_tune_cache_path",
           "SpwError", "SpwMatrix", "create_opts",
           "load", "spw_create", "spw_destroy", "spw_info", "spw_mv", "spw_vtm", "spw_mv_batch",
           "spw_vtm_batch", "spw_create_coo", "spw_cgls", "spw_plan_zones", "spw_round_values", "spw_profile_enable", "spw_profile_select",
           "spw_profile_reset", "spw_profile_read"]

"""MI355X reconstruction of cut quantum circuits (FD and DD, with entry
attribution) behind the C ABI in include/cutqc.h.  The Python layer only
marshals arguments; see ``api`` for the entry points."""
from .api import (attribute, cq_attribute, cq_autotune_enable, cq_label_balance_enable, cq_column_scaling_enable, cq_dd_lanes, cq_dd_checkpoint_bytes, cq_autotune_json, cq_autotune_load, cq_autotune_save, cq_plan_json, cq_profile_enable, cq_profile_read, cq_attribute_workspace_size, cq_dd_workspace_size,
                  cq_fd_workspace_size, cq_reconstruct_dd, cq_reconstruct_fd, cq_reconstruct_fd_noalloc,
                  cq_validate_cutmap,
                  cq_dd_bfs_workspace_size, cq_reconstruct_dd_bfs, cq_sample_shots,
                  cq_sample_shots_workspace_size, cq_chi2, cq_chi2_workspace_size,
                  cq_simulate_probabilities, cq_simulate_workspace_size, cq_variant_probabilities,
                  cq_variants_workspace_size, cq_find_cuts,
                  mask, reconstruct_dd, reconstruct_fd, validate_cutmap)
from ._lib import CQError, PRECISION

__all__ = ["attribute", "reconstruct_fd", "reconstruct_dd", "validate_cutmap", "mask",
           "cq_attribute", "cq_reconstruct_fd", "cq_reconstruct_fd_noalloc", "cq_reconstruct_dd", "cq_validate_cutmap",
           "cq_attribute_workspace_size", "cq_fd_workspace_size", "cq_dd_workspace_size",
           "cq_plan_json", "cq_label_balance_enable", "cq_column_scaling_enable", "cq_dd_lanes", "cq_dd_checkpoint_bytes", "cq_profile_enable", "cq_profile_read", "cq_autotune_enable",
           "cq_autotune_json", "cq_autotune_load", "cq_autotune_save", "cq_dd_bfs_workspace_size", "cq_reconstruct_dd_bfs", "cq_sample_shots",
           "cq_sample_shots_workspace_size", "cq_chi2", "cq_chi2_workspace_size",
           "cq_simulate_probabilities", "cq_simulate_workspace_size", "cq_variant_probabilities",
           "cq_variants_workspace_size", "cq_find_cuts", "CQError",
           "PRECISION"]

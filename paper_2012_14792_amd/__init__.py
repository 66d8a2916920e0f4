"""Dynamic tile + rectangular-slice (TRS) frame partitioning on AMD MI355X (gfx950).

The partitioning path (per-CTU features, predicted time map, prefix sums, exhaustive
two-step search) runs in the HIP kernels of libtrs.so; ``binding`` marshals arguments to
its C ABI (include/trs.h).
"""
from . import binding  # noqa: F401
from .binding import (Batch, Partitioner, TrsError, make_frame, make_params, read_result,  # noqa: F401
                      trs_partition,
                      trs_search_stats, trs_profile_enable, trs_profile_read,
                      trs_cost_map, trs_decode, trs_features, trs_release_plans, trs_search,
                      trs_search_workspace, trs_space_size)
from .binding import (trs_mlp_backward, trs_mlp_cost, trs_mlp_forward, trs_mlp_inputs)  # noqa: F401,E402

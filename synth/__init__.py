"""Seeded synthetic inputs for the batched cost-model path.

This package only draws numbers: model weights, per-stage pipeline features,
per-(stage, candidate) schedule features and cost terms, query sizes and
arrival times.  It holds none of the cost model's arithmetic, so both the
GPU path and the CPU oracle can take their inputs from here.
"""
from .workloads import (  # noqa: F401
    DIMS, PARAM_LAYOUT, N_PARAMS, WEIGHT_SEED,
    Query, Workload, model_params, unpack_params, draw_query, workload,
    ragged_sizes, serving_stream, f32_to_bf16_bits, bf16_bits_to_f32,
)

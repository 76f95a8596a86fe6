"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package holds no arithmetic of the clustering method.  It produces:

* datasets shaped like the workloads the paper clusters (``datasets``);
* the random draws the method consumes (landmark sets, k-means++ uniforms,
  random initial labels) from a counter-based generator written from its
  published definition (``rng``), so that the oracle and the HIP library can
  both be handed the same draws, or each reproduce them independently.
"""
from . import rng, datasets  # noqa: F401
from .rng import (  # noqa: F401
    SplitMix64, stream, landmark_count, draw_landmarks, draw_all_landmarks,
    draw_kmpp_uniforms, draw_init_labels, batch_index_sets,
    PURPOSE_LANDMARKS, PURPOSE_INIT_LABELS, PURPOSE_KMEANSPP, PURPOSE_SUBSAMPLE,
)

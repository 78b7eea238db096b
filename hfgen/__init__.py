"""Seeded synthetic inputs shared by the product tests, the benchmark and the
oracle's tests.  Holds no arithmetic of the method itself."""

from .configs import CONFIGS, CUT_KINDS, RECO_DEFAULTS, config, default_order, dep_masks  # noqa: F401
from .events import generate, stream_chunk, subset  # noqa: F401

"""MI355X (gfx950) hot path of a HEP-Frame-style analysis (arXiv:2211.14346):
cut chain with adaptive ordering, on-device compaction and the dileptonic
ttbar kinematic reconstruction, behind the C ABI in include/hf.h."""

from . import binding  # noqa: F401
from .binding import HFError, lib  # noqa: F401

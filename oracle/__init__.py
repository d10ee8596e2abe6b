"""FP64 CPU oracle (test infrastructure only; see render.py)."""
from .render import *  # noqa: F401,F403

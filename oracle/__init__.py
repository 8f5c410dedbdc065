"""Plain FP64 CPU oracle (test infrastructure only; see mercer_gp)."""
from .mercer_gp import *  # noqa: F401,F403

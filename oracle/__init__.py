"""FP64 CPU oracle (test infrastructure only; see ``kaze_oracle``)."""
from .kaze_oracle import *  # noqa: F401,F403
from .kaze_oracle import __all__  # noqa: F401

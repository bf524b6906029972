"""CPU oracle (test infrastructure only): a plain FP64 numpy implementation of
the low-rank splitting schemes, used to check the HIP path.  The product path
never imports this package."""
from .dme_oracle import *  # noqa: F401,F403

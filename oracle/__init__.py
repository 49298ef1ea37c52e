"""CPU FP64 oracle of the Elfpie iteration (test infrastructure only; see elfpie_oracle)."""
from .elfpie_oracle import *  # noqa: F401,F403
from . import elfpie_oracle  # noqa: F401

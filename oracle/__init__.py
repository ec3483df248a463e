"""CPU FP64 oracle (test infrastructure only; shares no code with the GPU library)."""
from .soar_oracle import *  # noqa: F401,F403
from .philox import philox4x32_10, philox_uniform24, philox_index  # noqa: F401

"""CoNet-Rx on AMD Instinct MI355X: gfx950 HIP kernels behind a C ABI (libconet.so).

The Python layer only marshals arguments; see binding.Conet.
"""
from .binding import (Conet, ConetError, Server, conet_function, featurise, load, make_config, mfma_dot, mfma_peak,
                      pinned_array, simulate, weight_count,
                      workspace_bytes, EXPORTS)

"""MI355X-native checkerboard Metropolis engine for the thin-film Ising model
of arXiv:1411.5588 (HIP kernels behind the C ABI in include/islf.h)."""
from .islf import (APBC, BITPACK, EXEC_BATCHED, EXEC_PERSISTENT, EXEC_PLAIN, GAPBC, INIT_DOWN,  # noqa: F401
                   INIT_HOST, INIT_RANDOM, INIT_UP, INT8, PBC, Context, IslfError, Replica,
                   energy, footprint_bytes, integrate, integrate_device, num_tiles)

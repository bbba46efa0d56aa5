"""MI355X (gfx950) SMC sampler with a ChEES-HMC proposal.

The sampler runs in hand-written HIP kernels behind the C ABI declared in
include/chees_smc.h (libchees_smc.so).  `paper_2504_02627_amd.chees` is the thin
ctypes binding; importing this package does not load the library.
"""

__all__ = ["chees", "synth", "build"]

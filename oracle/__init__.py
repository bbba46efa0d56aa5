"""Oracle: a plain, slow, binary64 CPU implementation of SMC with a ChEES-HMC
proposal, written from the paper (arXiv 2504.02627).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call, link
or execute anything under this directory; only the tests, the smoke check and
the CPU-baseline leg of the benchmark do.  It shares no code with the device
library and the library never imports it.
"""

from . import philox, smc  # noqa: F401

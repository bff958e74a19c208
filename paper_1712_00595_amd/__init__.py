"""MI355X dynamic random walk with restart: offset score propagation (OSP /
OSP-T) behind a C ABI (``include/rwr.h``), implemented by HIP kernels for
gfx950 in ``csrc/`` and exposed to Python by :mod:`.rwr`."""

from .rwr import EXPORTED, Context, RwrError, load_library  # noqa: F401

"""MI355X (gfx950) triangular-matrix inverse by recursive 2x2 splitting.

Python entry points over the C ABI of libtrinv (include/trinv.h). The HIP
library must be built (``paper_2307_07611_amd/build.py``); importing the
package works without it, but every call then raises.
"""

from ._lib import MODES, TrinvError, load  # noqa: F401


def __getattr__(name):
    # The torch-facing wrappers import torch lazily so that the ABI checks can
    # run without it.
    import importlib

    if name.startswith("__"):
        raise AttributeError(name)
    api = importlib.import_module(__name__ + ".api")
    if hasattr(api, name):
        return getattr(api, name)
    raise AttributeError(name)

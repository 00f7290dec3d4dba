"""Block belief propagation for 2D PEPS on MI355X (gfx950).

The computation lives in the HIP library ``libbbp.so`` behind the C ABI of
``include/bbp.h``; :mod:`paper_2301_05844_amd.bbp` is its ctypes binding.
"""


def __getattr__(name):
    if name in ("BlockBP", "BBPError"):
        from . import bbp
        return getattr(bbp, name)
    raise AttributeError(name)

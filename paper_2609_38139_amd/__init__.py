"""MI355X-native local autonomous inference machine decoder for quantum LDPC codes.

The decoder runs many Monte-Carlo shots at once: belief propagation on the
Tanner graph of H_X interleaved with belief-guided local moves of the active
syndrome checks. The compute path is hand-written HIP for gfx950 behind a
C ABI (``include/laim.h``); :mod:`paper_2609_38139_amd.laim` is the thin
Python binding. :mod:`paper_2609_38139_amd.codes` builds the code families.
"""

__all__ = ["codes", "laim"]


def __getattr__(name):
    if name in ("codes", "laim"):
        import importlib
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)

"""MI355X-native steady and transient chip-temperature solve (VarSim, arXiv 2307.12119).

The compute path is the HIP library ``libvarsim.so`` built from ``csrc/`` (see ``build``);
``varsim`` is its ctypes binding.  Importing the package loads nothing: call
``varsim.Library.load()`` or create a ``varsim.Context``.
"""

__all__ = ["build", "varsim"]

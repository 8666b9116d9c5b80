"""MI355X-native lattice Boltzmann hot path (arXiv 2512.12213).

The compute path is the HIP library ``liblbm.so`` (C ABI in include/lbm.h);
``lbm`` is its ctypes binding and ``workloads`` holds the synthetic workload
definitions and seeded input generators.
"""
import importlib

from . import workloads  # noqa: F401


def __getattr__(name):
    if name in ("lbm", "Lattice", "from_workload"):
        mod = importlib.import_module(__name__ + ".lbm")
        return mod if name == "lbm" else getattr(mod, name)
    raise AttributeError(name)

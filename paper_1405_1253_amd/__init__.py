"""MI355X-native D2Q37 thermal lattice Boltzmann hot path.

The method is the thermal LBM of Ripesi, Biferale, Schifano and Tripiccione,
Phys. Rev. E 89, 043022 (2014): one fused time step (pull streaming, wall
rows, force-shifted BGK collision with a 4th-order Hermite equilibrium) on a
lattice periodic in x with thermal walls in z, plus the three-layer
Rayleigh-Taylor initial state and its diagnostics.

The computation lives in liblbm.so (hand-written HIP for gfx950, C ABI in
include/lbm.h); ``abi`` binds it under the same names and ``runtime.Lattice``
manages the device buffers.  ``workload`` holds the seeded synthetic inputs.
"""
from . import workload  # noqa: F401  (no GPU or library needed)


def __getattr__(name):
    # the binding loads liblbm.so lazily so that workload stays importable
    if name in ("abi", "runtime", "Lattice"):
        import importlib
        mod = importlib.import_module(f".{'runtime' if name == 'Lattice' else name}", __name__)
        return mod.Lattice if name == "Lattice" else mod
    raise AttributeError(name)

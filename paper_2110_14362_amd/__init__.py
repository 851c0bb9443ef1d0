"""Random batch Ewald (RBE) Fourier-space step for periodic NPT charge systems on
AMD Instinct MI355X (gfx950).

The compute path is the HIP library ``librbe.so`` (C ABI in ``include/rbe.h``);
:mod:`paper_2110_14362_amd.rbe` is its thin ctypes binding and
:mod:`paper_2110_14362_amd.workloads` holds the seeded synthetic inputs.
Importing this package loads nothing; the library is loaded on first use and
its absence is an error, never a fallback.
"""

__all__ = ["rbe", "workloads", "build"]

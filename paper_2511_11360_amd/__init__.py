"""MI355X-native phase-field lattice Boltzmann hot path.

The compute path is the HIP library ``libpflbm.so`` built from ``csrc/``; the
Python modules only marshal arguments to its C ABI (``pflbm``), manage device
buffers and streams through PyTorch (``solver``) and orchestrate the adjoint
time loop (``autograd``). ``workloads`` builds seeded synthetic inputs.

Importing the package loads nothing native; the library is loaded on first use
and a missing library raises instead of falling back to any other path.
"""

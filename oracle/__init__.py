"""FP64 CPU oracle of the lattice Boltzmann step (test infrastructure only).

Only ``tests/``, the smoke check in ``__graft_entry__`` and the CPU-baseline
leg of ``bench.py`` may import this package. It shares no code with the HIP
library and never imports it.
"""

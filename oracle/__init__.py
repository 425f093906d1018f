"""CPU oracle for the NFFT hot path -- TEST INFRASTRUCTURE ONLY.

* ``oracle.ndft``     FP64 direct NDFT and adjoint (C + OpenMP via ctypes): the
  exact transform the NFFT approximates.
* ``oracle.nfft_alg`` plain FP64 NFFT following the paper's Algorithms 1 and 2
  step by step (numpy), the oracle for the GPU path's results.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import, call or execute anything in this package.  The GPU
library and its Python binding never do.
"""

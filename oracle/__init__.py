"""CPU oracle for softened self-gravity -- TEST INFRASTRUCTURE ONLY.

Plain, slow, FP64 reference implementations written from the paper
(arXiv 2010.11254, Sec. 2.2 "Gravity" and Sec. 2.2.1 "Softening"):

* ``oracle.direct``: O(N^2) direct sum (C + OpenMP), its exact adjoint and a
  pair-local loss for finite differences;
* ``oracle.tree``: a Barnes-Hut octree with the same keys, topology, groups,
  opening decisions and multipole evaluation the GPU tree path is specified
  to produce, evaluated in FP64 with torch so that autograd gives the adjoint
  of the frozen-list approximation.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library does not link, call or
share code with it.
"""

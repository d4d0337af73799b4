"""CPU FP64 oracle for the block-AMR Euler cycle: TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package. It shares no code with the GPU library
(``paper_2202_12309_amd``) and imports nothing from it.

* ``pkh_oracle.c`` (wrapped by :mod:`oracle.oracle`): the block mesh, ghost
  fill with restriction/prolongation, flux correction, VL2 cycle, CFL
  timestep, conserved totals and regridding, written from the method's
  definition.
* :mod:`oracle.torch_ref`: an independent uniform-periodic-grid formulation in
  plain PyTorch CPU FP64 ops (no blocks, no ghosts: neighbours by
  ``torch.roll``). It cross-checks the C oracle and, through autograd, is the
  reference gradient for the adjoint.
* :mod:`oracle.exact_riemann`: the exact Riemann solution of the ideal-gas
  Euler equations (Toro, ch. 4), used to pin the shock-capturing result.
"""

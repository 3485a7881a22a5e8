"""Oracle: a plain, slow FP64 CPU implementation of the transformer
density-operator hot path (arXiv 2502.20723).

THIS PACKAGE IS TEST INFRASTRUCTURE. Only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` may import it. The product path
(the HIP library and its Python binding) never imports, calls or links it, and
it shares no code with that path: the two meet only through the seeded input
generators, which hold none of the method's arithmetic.

Modules (each function cites the passage of the paper it follows):

* ``lindblad``  - the vectorised GKSL generator (Eq. VecLin, App. A) of the
                  dissipative Ising and XYZ chains, evaluated row by row from
                  the local operator matrices.
* ``ansatz``    - the transformer density operator (main text "Transformer
                  density operator ansatz", App. B) and its parameter layout.
* ``vmc``       - the local Lindbladian estimator, the cost (Eq. lossnetk) and
                  its gradient (App. C, "Optimization Procedure").
* ``philox``    - the Philox4x32-10 counter-based generator (Salmon et al.,
                  SC'11), from its published definition.
* ``sampler``   - Metropolis-Hastings on |rho|^2 (App. C, "Efficient Sampling
                  Strategy").

Parity status of each function is stated in its module header; the network
forward has no printed values to pin to and is pinned by invariants and by
independent library re-derivations (see tests/test_oracle_ansatz.py).
"""

"""fp64 CPU oracle of the dSMC smoother (Corenflos, Chopin, Sarkka, 2022).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or links
this package: only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline
leg of ``bench.py`` may use it.  It shares no code with the HIP path; the two
meet only through the seeded synthetic inputs of
``paper_2202_02264_amd/workloads.py`` (which this package never imports) and
through the Philox4x64-10 stream layout, which each side implements on its own
from the generator's published definition.

Modules:
  philox   Philox4x64-10 counter-based generator and the uniform / normal draws
  ssm      model log densities (prior, transition, potential, proposal)
  dsmc     Algorithm 2 (leaves), Algorithm 1 (combine), Algorithm 6 (tree),
           conditional dSMC (Section 3.1, Algorithm 4)
  kalman   Kalman filter / RTS smoother / exact log-likelihood (closed-form pins)

Parity pins for each function are in tests/test_oracle_*.py.
"""
from . import dsmc, kalman, philox, ssm  # noqa: F401

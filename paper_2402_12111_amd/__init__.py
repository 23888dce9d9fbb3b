"""MI355X (gfx950) Heston Monte Carlo / Longstaff-Schwartz hot path of the SIMR
market-risk benchmark (Klaisoongnoen et al., FPGA'24).

Every step of the path runs in hand-written HIP kernels inside ``libsimr.so``
behind the C ABI of ``include/simr.h``; this package only marshals arguments
(:mod:`paper_2402_12111_amd.simr`) and holds the seeded input recipes
(:mod:`paper_2402_12111_amd.workloads`).  Importing the package does not load
the library; the first call into :mod:`.simr` does, and it raises if the library
is missing or no GPU is present.
"""

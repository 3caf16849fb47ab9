"""MI355X (gfx950) HIP implementation of the EE2 exponential-Krylov and LIM
Chebyshev time steps for the periodic Cahn-Hilliard equation
(Botchev, arXiv 2502.14589).  The compute path is libch.so (include/ch.h);
`ch` is its Python binding and `inputs` the seeded synthetic workloads.
"""

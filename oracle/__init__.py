"""FP64 CPU oracle for the masked Gross-Pitaevskii solver (test infrastructure).

This package is test infrastructure: only the test-suite, the smoke check
and the CPU-baseline leg of the benchmark may import it.  The product path
(the HIP library and its Python binding) never calls into it.

It is a plain, slow, obviously correct restatement of what the paper
computes, in float64 / complex128, with no blocking, fusion or reordering
beyond what the paper's own equations state:

* operator.py     reduced kinetic operator T~ (Sec. II.A, App. B eq. (B1)),
                  built two independent ways;
* potential.py    RF-dressed potential eq. (10) with a piecewise-linear
                  detuning ramp (Sec. V);
* observables.py  particle number eq. (3), energy and chemical potential;
* itp.py          imaginary-time split step with renormalisation (Sec. II.A,
                  eqs. (6)-(7));
* realtime.py     classic RK4 on eq. (8) (Sec. II.A), in k-form;
* dense.py        dense Cartesian brute force with the region of interest
                  applied as a projector;
* adjoint.py      discrete adjoint of the RK4 map for a fidelity loss with
                  respect to ramp knots, with sqrt(N) checkpointing (the
                  paper is silent here; see the module docstring);
* tableau.py      the memory-optimised Runge-Kutta coefficients of App. A,
                  derived in exact rational arithmetic;
* restage.py      staged ramps of Sec. V: potentials interpolated linearly
                  between stage arrays, re-post-selection at each stage end
                  and the carry-over of psi between grids.

Units: hbar = m = 1, so T~ = -1/2 Laplacian restricted to the active set.
"""

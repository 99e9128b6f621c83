"""Plain, slow CPU reference ("oracle") of the coupled phase-field lattice
Boltzmann step: test infrastructure only.

Only the test-suite, the smoke check and the CPU-baseline leg of the benchmark
import this package. The product path (the HIP library and its Python
binding) never imports, calls or links anything here, and nothing here
imports the product package.

Every routine works on numpy arrays in float64, or complex128 when a
complex-step derivative is taken, and follows the paper's equations in the
paper's order (Li, Zhang, Wu, Peng, Wang, "Comparative study and critical
assessment of phase-field lattice Boltzmann models ...", arXiv 2511.11360).

Naming. The paper calls the phase-field distribution g_alpha and the
hydrodynamic one f_beta (Sec. II.B, Eq. fakhari_model_simplified). This package
and the library use g = hydrodynamic distribution (paper's f) and h = phase-field
distribution (paper's g); W is the paper's interface width xi and M its
mobility M_phi.
"""

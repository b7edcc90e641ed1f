"""Plain FP64 CPU oracle for the Chebyshev-filtered plane-wave eigensolver path.

TEST INFRASTRUCTURE ONLY.  Only the tests, ``__graft_entry__.smoke()`` and the
bench's ``cpu_baseline`` leg may import this package; the product path (the HIP
library and its Python binding) never calls it and shares no code with it.

Each function follows a passage of the paper (arXiv 2604.11139): the problem
statement H psi = lambda S psi (section "Problem setup"), with S = I or the
projector overlap S = I + P Q P^H and its Woodbury inverse (module overlap), the
matrix-free Hamiltonian with FFT local part and projector nonlocal part
(sections "Main computational kernels" and "Low-level operations"), the
Chebyshev spectral filter with Rayleigh-quotient bounds (Algorithm
"Parallel Chebyshev filtering of degree k" in the appendix on parallel
subspace iteration algorithms), S-orthogonalisation by Cholesky (Algorithm
"S-ortho") and the Rayleigh-Ritz procedure (Algorithms "Rayleigh-Ritz
procedure" / "Matrix-free Rayleigh-Ritz procedure").  Where the paper is silent
the module docstrings state the reading taken.

Everything is written in float64 / complex128 with NumPy and SciPy; library
primitives (FFT, dense eigensolver, Cholesky) are used as single steps, never
blocked, fused or reordered.
"""
from .sphere import GSphere, gsphere, reciprocal_vectors  # noqa: F401
from .hamiltonian import Hamiltonian, density  # noqa: F401
from .chebyshev import (  # noqa: F401
    cheb_filter,
    cheb_sigmas,
    filter_bounds,
    lanczos,
    lanczos_upper_bound,
    rayleigh_quotients,
)
from .subspace import (  # noqa: F401
    cholesky_upper,
    gram,
    rayleigh_ritz,
    residual_norms,
)
from .adjoint import filter_backward, filter_coefficients, filter_iterates, filter_loss  # noqa: F401,E402
from .overlap import (  # noqa: F401,E402
    Overlap,
    filter_bounds_gen,
    lanczos_gen,
    lanczos_upper_bound_gen,
    rayleigh_quotients_gen,
    rayleigh_ritz_gen,
    residual_norms_gen,
    sinv_h,
)
from .lobpcg import lobpcg_pass, tpa_precondition  # noqa: F401,E402
from .scf import hartree, lda_exchange, mix, occupations, scf_iteration, scf_potential  # noqa: F401,E402

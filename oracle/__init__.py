"""FP64 CPU oracle for the Maxwell parallel imaging encoding operator.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or
links this package: only the test suite, the smoke check and the CPU
baseline leg of the benchmark use it.  It is a plain, slow, obviously
correct NumPy implementation written from the paper (Francavilla et al.,
"Maxwell Parallel Imaging"), in float64 / complex128, with no blocking,
fusion or reordering beyond what the definitions state.  It shares no code
with the HIP path; both only consume the seeded inputs of ``synth``.

Modules
-------
dft       centred unitary DFT (Sec. II-A, the operator F_s; Sec. II-B, the DFT matrix)
basis     dense and Tucker basis apply and adjoint (Sec. II-B Eq. (5); Sec. II-E)
nufft     Kaiser-Bessel NUFFT type 2 / type 1 and the exact NDFT (Sec. III-B, radial F)
encoding  encoding operator, Jacobian adjoint, JVP, loss and gradient (Sec. II-B)
solver    Gauss-Newton normal operator and conjugate gradients of the IRGN step (Sec. II-B, Eq. (6))
admm      SENSE with fixed maps, ball projection, TV prox and the constrained ADMM (Sec. II-C)
compress  accuracy-controlled Tucker compression of a dense basis by ST-HOSVD (Sec. II-E)

Every public function is pinned by ``tests/test_oracle_pins.py`` and
``tests/test_oracle_solver.py``, ``tests/test_oracle_admm.py`` and
``tests/test_oracle_compress.py`` against
brute force, closed forms, invariants or library special cases.
"""
from .dft import centred_dft, centred_idft  # noqa: F401
from .basis import (dense_apply, dense_adjoint, mode_product, tucker_coil_map,  # noqa: F401
                    tucker_apply, tucker_adjoint, tucker_materialise)
from .nufft import (kb_beta, kb_kernel, kb_deapod, nufft_type2, nufft_type1,  # noqa: F401
                    ndft, ndft_adjoint)
from .encoding import Oracle  # noqa: F401

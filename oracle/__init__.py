"""Plain FP64 CPU oracle for the neural-constitutive finite-element hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library, its
Python binding) may import, call or link anything in this package; only the
test suite, the smoke check and the CPU-baseline leg of the benchmark do.

The oracle is written from the paper (COMMET, arXiv 2510.00884) and shares no
code with the GPU path.  It evaluates the plain definitions, vectorised over
quadrature points with NumPy, in the paper's order:

* ``ncm``      kinematic layer (invariants, App. A.2.1-A.2.2; training features,
               App. C), inner network of eq. icnn with its input gradient (reverse
               sweep) and input Hessian (Hessian-vector products), stress and
               stiffness by the push-forward route
               (eqs. stress-cgo, stiffnes-cgo, second-and-fourth) pulled back to
               P and dP/dF (App. A.1).
* ``fe``       isoparametric hex8 / tet10 elements, Gauss quadrature, element
               residual and stiffness in the paper's spatial form
               (eqs. apprx-k, apprx-r, r-quad, k-quad; Alg. 2) and global
               assembly (node-major dof order of Sec. 2.1).
* ``calib``    stress-calibration loss and its parameter gradient, by PyTorch
               reverse-mode AD on the CPU in FP64.

Readings of the paper where it is silent or misprinted are listed in the
module docstrings of ``ncm`` and ``fe``.  Every function is pinned by the
``-m "not gpu"`` tests in ``tests/test_oracle_*.py``.
"""

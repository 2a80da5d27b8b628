"""CPU oracle for MatExPre (complex128, NumPy/SciPy).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
link anything in this package; only the tests, the smoke check and the
benchmark's CPU-baseline leg use it.  It shares no code with the GPU library:
it assembles its own sparse matrices, evaluates matrix functions with library
routines (dense expm, the Al-Mohy--Higham expm_multiply) and runs its own
GMRES / FGMRES in the order the paper states them.

Modules
-------
operator  -- absorbing-layer finite-difference Helmholtz matrix A, the shifted
             A_s = A + i omega^2 s D, right-hand side b = -f.
matfun    -- psi functions, exp(itA_s)v and psi_1(itA_s)v, closed forms.
krylov    -- GMRES / FGMRES, the preconditioner M(r) of Algorithm 1, direct solve.
conv      -- reference 3x3x3 convolutions for the learned stage.

Parity status per function is listed in each module's header.
"""

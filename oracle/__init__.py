"""FP64 CPU oracle for the gDC Brownian-dynamics step with fluctuating FCM.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and
its Python binding) may import, call or link anything in this package; only
``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` use it.  It shares no code with the GPU path: it re-derives every
step from the paper (Westwood, Delmotte & Keaveny, "A generalised
drift-correcting time integration scheme for Brownian suspensions of rigid
particles with arbitrary shape", arXiv 2106.00449) in plain NumPy/SciPy,
FP64 throughout, written for readability rather than speed.

Modules
-------
quaternion  Appendix A: rotation matrix, Hamilton product, exp map, dexpinv.
philox      Philox4x32-10 (Salmon et al., SC'11) and the Box-Muller normal
            transform with its own log/sin/cos series (the noise contract).
fcm         Sec. 4.2: Gaussian spreading S, averaging J = S*, the spectral
            Stokes solve L^-1 and M_FCM = J L^-1 S.
noise       Sec. 4.2 / Sec. 6.1: the fluctuating stress and the random
            velocity field, in the Fourier-space (canonical) and the
            real-space (as printed) forms.
rigid       Sec. 2.2: the rigid-body map K, K^T K, the least-squares
            velocity, the saddle-point mobility problem, GMRES with the
            block-diagonal preconditioner, the body mobility N.
gdc         Sec. 3: the gDC step (finite-difference and RFD divergence),
            Appendix D: the Euler-Maruyama step, and the force models.

Every function with a pin (a closed form, an invariant, a brute-force
evaluation, a published test vector or a statistical law) is checked by the
``-m "not gpu"`` tests.  Functions without such a pin say "parity unpinned".
"""

from . import quaternion, philox, fcm, noise, rigid, gdc  # noqa: F401

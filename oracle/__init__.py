"""Plain FP64 CPU oracle for the FFT-CG boundary element method of
Li & Popov, "Boundary element method for normal non-adhesive and adhesive
contacts of power-law graded elastic materials" (arXiv:1612.08395).

THIS PACKAGE IS TEST INFRASTRUCTURE.  It exists to prove the GPU library
right, not to compute results for users.  Only the test suite, the smoke
check in ``__graft_entry__`` and the ``cpu_baseline`` leg of ``bench.py`` may
import it.  The product path (``paper_1612_08395_amd``) never imports,
links or calls anything here, and nothing here imports the product path.

Everything is written for a reader holding the paper: each function cites
the section / equation it follows and is plain, slow and obviously correct
(numpy / scipy in float64, no blocking, fusion or reordering beyond what the
cited definition states).

Modules
-------
material    alpha, beta (Eqs. 3-4), compliance prefactor (Eq. 2/12),
            Table 1 corrected c1 and its interpolation, Eq. 23 c1, p_crit (Eq. 24)
influence   influence coefficients by quadrature of the point-force
            solution over one rectangular element (Eqs. 8-10)
convolution direct O(N^4) sum (Eq. 7) and zero-padded FFT form (Eq. 13)
solver      constrained conjugate-gradient contact solve (Section 2.1, the
            method the paper cites for the inverse problem) and the adhesive
            detach / re-solve loop (Section 3.1)
analytic    closed forms used only as pins (Eqs. 11, 14-17, 25-26 and the
            readings derived from them)

Parity status of each function is stated in its module header.
"""

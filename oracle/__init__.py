"""Plain FP64 CPU oracle for the steady and transient temperature solve.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or run anything in this package.  The GPU
library never calls it and shares no code with it; the two meet only in the seeded inputs
of the ``workloads`` package.

Modules
-------
kernel     cell-averaged Green's function of the die (Sec. II-B, Appendix Theorem I), the
           method of images for the die edges (Sec. IV-F)
stack      Green's function of a layered package (Table param) with an isothermal or convective
           bottom: the first layer's image series plus the cosine series of the stack's extra
           impedance
steady     direct spatial summation and the leakage / conductivity fixed point
           (Eqs. Pt, Pleak, condsi, fspvsk; the iterate-to-convergence ground truth of Sec. V-C)
anderson   Anderson(1)-accelerated iteration of the same fixed point (a classical baseline,
           not from the paper)
oneshot    one-shot leakage-aware modified Green's functions, deterministic and random parts
           (Sec. IV-C: Eqs. detsol, randsol, detrandsol) in a well-posed discrete reading
transient  single-pole transient Green's function (Eq. tranGreen) and full-history
           superposition of step responses (Eq. tranapprox)
fd         brute-force finite-volume solve of the heat equation (Eq. fourier), used to pin
           the kernel to the physics (single slab, laterally varying k, layered box)
surrogate  FP64 reference layers of the convolutional warm-start network

Parity status of each function is stated in its module header.
"""

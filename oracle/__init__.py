"""Plain FP64 CPU oracle for the two-stage separable blob-detection filter bank
of H. L. Kennedy, "Digital filters with vanishing moments for shape analysis"
(arXiv:1912.07133).

THIS PACKAGE IS TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` may import or call it.  The product
(``paper_1912_07133_amd``, its C-ABI library and HIP kernels) never imports,
links or executes anything here, and this package imports nothing from the
product: the two share no kernels, helpers, tables or constant generators.

Everything is written for a reader holding the paper, in its order and
notation, in float64 (or arbitrary precision for the design step), with no
blocking, fusion or reordering beyond what the paper states:

* ``design``    -- filter design: the repeated-pole IIR blur of Section 4.3
                   (Table IV closed form and the general constrained procedure
                   of Eqs 12-15, 23-24), the three-term decomposition of
                   Eqs A11-A19, the coloured Savitzky-Golay FIR of Section 4.2
                   (Eqs 20-22), the sampled Gaussian of Eqs 9 and 11, the
                   interpolating differentiators of Table I, the Butterworth
                   blur of Section 4.4 / Eqs A26-A31.
* ``filtering`` -- the three-term difference equation (Eqs A6-A10) with the
                   steady-state initialisation of Eq A32, the FIR convolution
                   of Eq A5, separable x-then-y application (Sections 2 and 5),
                   and a brute-force 2-D convolution for tiny images.
* ``shape``     -- the high-pass stage (Table I taps), the scale-normalised
                   Laplacian, the multi-scale strict-extremum blob list, and the
                   Hessian detector of Eqs 26-27.

Parity status of each function is stated in its docstring; every function is
pinned by a ``-m "not gpu"`` test except where the docstring says
"parity unpinned".
"""

from . import design, filtering, shape  # noqa: F401

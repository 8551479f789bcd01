"""Plain FP64 CPU oracle for the time-dependent weighting field and Eq. 1.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path may import it: only the
test suite, the smoke check of the package entry file and the CPU-baseline leg
of the benchmark call into this package.  It shares no code with the HIP path
(no kernels, headers, tables, constants or helpers) and imports nothing from it.

What it computes (paper: abstract, Eq. 1 in the introduction, Section 3):

* ``green``       the periodic, band-limited, Gaussian-smoothed potential G and
                  field E_G = -grad G of a unit charge in the diamond, as direct
                  sums over the discrete mode set (the fundamental solution that
                  Section 3 translates and rescales).
* ``collocation`` the fundamental-solution boundary fit: point charges on the
                  column axes whose magnitudes are fixed, at each frequency, by
                  matching the diamond potential on the column surface to the
                  potential inside the resistive column (an RC line), plus
                  charge neutrality and a gauge constant.
* ``timegrid``    the real inverse Fourier quadrature from the frequency grid to
                  the time samples (convention exp(+i w t)).
* ``field``       H(x, t) on the grid, three independent ways: direct
                  superposition of translated fundamental solutions (tiny grids),
                  a full 3D inverse FFT, and direct per-column sums (sampled
                  columns of large grids).
* ``convolution`` Eq. 1 discretised per carrier step: midpoint position,
                  displacement for v dt', rectangle rule in the lag, trilinear
                  interpolation of the grid field with periodic wrap.
* ``electronics`` the currents convolved with a front-end impulse response,
                  plus noise, and per-track timing features (amplitude, peak
                  time, constant-fraction time).
* ``timedomain``  the paper's own forward-Euler time stepping of the boundary
                  charges on the same RC-line model, as a cross-check of the
                  frequency-domain solve.
* ``gradient``    forward-mode derivatives of the currents with respect to each
                  column's quarter-column resistivities and radius: the
                  derivative of the boundary-fit system, solved per frequency,
                  pushed through the linear rest of the path.

Pins (tests marked "not gpu"): Ewald sums for G and E_G; the direct G against
the nested collocation sums; the compact RC-line system against a Kirchhoff
(KCL + Ohm) assembly; LU against QR with backward error; static potentials at
zero frequency; the electrode-sum rule; the full-period identity of the time
quadrature; the textbook Ramo-Shockley limit for perfectly conducting columns;
passivity and causality; the three field routes against each other; charge
conservation of the convolution; brute-force loops for the convolution; the
closed-form convolution of two sampled exponentials, the identity response,
a sampled parabola's vertex and a linear ramp's constant-fraction crossing for
the electronics; for the time-domain scheme, its transfer function against
the collocation system, its zero- and infinite-time limits, and first-order
convergence of forward Euler to the exact step response; for the derivatives,
central differences of the whole forward pipeline and of the collocation
matrix, and the common conductivity derivative of parallel quarter-columns.

Parity unpinned: none of the computed quantities.  The modelling readings
themselves (thin-wire columns, smoothing widths, periodic z, collocation
azimuth, column permittivity) are choices, not results, and are not pinned.
"""
from . import green, collocation, timegrid, field, convolution, electronics, timedomain, gradient  # noqa: F401
from .pipeline import weighting_field, induced_current  # noqa: F401

"""Time-dependent weighting field H(x, t) and Eq. 1 induced currents on MI355X.

Submodules:
  wt         ctypes binding of the HIP library (include/wt.h); loads libwt.so
  workloads  seeded synthetic inputs (geometry, spectra, carrier paths)
  layout     index helpers for the time-blocked H layout
  build      builds libwt.so for gfx950

Importing the package itself loads nothing; ``from paper_2605_13987_amd import wt``
loads the library and raises if it has not been built.
"""

"""Independent FP64 CPU oracle for the coherent F-statistic search.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and its
Python binding) may import, call, link or execute anything in this package.  It
is used by ``tests/``, by the smoke check in ``__graft_entry__`` and by the
``cpu_baseline`` leg of ``bench.py`` -- nowhere else.

The oracle is written from the paper (Astone, Borkowski, Jaranowski, Krolak,
Pietka, "Data analysis of gravitational-wave signals from spinning neutron
stars. V. A narrow-band all-sky search"):

* ``model``  -- detector geometry, the Roemer delay n0.r_d/c (Sec. II, Eqs.
  pha3-pha5), amplitude-modulation functions a(t), b(t) (Sec. II), and the
  signal model used for injections (Eqs. resp, patt, hphc, h0iota, sig).
* ``method`` -- the resampled F-statistic of Sec. VI (Eqs. pham/phas, Bt, ia,
  DFT), the exact F-statistic by direct summation (Eqs. OS, Fab), the
  continuous-frequency variant and its analytic gradient.
* ``sums``   -- the plain C summation loops (direct DFT at chosen bins, direct
  matched-filter sums), OpenMP over output bins, Neumaier-compensated.

Everything is plain and slow on purpose: no blocking, fusion or reordering
beyond what the definitions state.  No code is shared with the HIP path.
"""

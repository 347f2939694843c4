"""Patchy semi-Lagrangian solver for the minimum-time HJB equation on MI355X.

The compute path is the C-ABI library ``libhjb.so`` (hand-written HIP for
gfx950); :mod:`paper_1109_3577_amd.hjb` is its thin Python binding and
:mod:`paper_1109_3577_amd.problems` the seeded problem generators.
"""

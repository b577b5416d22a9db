"""Preconditioned orbital minimization (OMM) for planewave Hamiltonians on MI355X.

The compute path lives in the HIP/C-ABI library ``libpomm.so`` (sources in
``csrc/``, declarations in ``include/pomm.h``); :mod:`.pomm` is its thin Python
binding.  :mod:`.inputs` generates seeded synthetic workloads.  Importing this
package loads nothing native; ``from paper_1603_09724_amd import pomm`` does.
"""

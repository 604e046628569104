"""MI355X-native relaxing-TVD + constrained-transport ideal-MHD time step.

The compute path is the HIP library built from ``csrc/`` (C ABI declared in
``include/mhd.h``); ``binding`` is its thin ctypes binding and ``problems``
builds synthetic initial states.
"""

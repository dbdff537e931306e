"""MI355X-native Monte Carlo assembly of the PDDSparse interfacial system G u = b.

The compute path is the HIP library ``libpdd.so`` (built from ``csrc/``),
reached through the thin ctypes binding in ``pdd``.  ``workloads`` holds the
seeded synthetic inputs.
"""

"""MI355X-native engine for the functionalized Cahn-Hilliard gradient flow.

The compute path is the HIP library ``libfch.so`` built from ``csrc/``; the
ctypes binding in :mod:`paper_2006_04784_amd.fch` loads it on first use and
raises if it is missing.  :mod:`paper_2006_04784_amd.inputs` holds the seeded
initial-state generators.
"""

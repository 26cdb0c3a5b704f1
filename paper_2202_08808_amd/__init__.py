"""Batch-dynamic SpGEMM on AMD MI355X (gfx950).

``dsg`` is the binding of the HIP library ``libdsg.so`` (C ABI in
``include/dsg.h``); ``inputs`` draws the seeded synthetic workloads.
"""

"""MI355X-native dynamically screened ISTA/FISTA for the Lasso and the Group-Lasso.

The compute path is the HIP library ``libdynscreen.so`` (built from ``csrc/``),
reached through the C-ABI declared in ``include/dynscreen.h``.  The Python
binding ``paper_1412_4080_amd.binding`` only marshals arguments; importing it
raises if the library is missing.  ``paper_1412_4080_amd.datagen`` draws the
synthetic inputs and needs no GPU.
"""

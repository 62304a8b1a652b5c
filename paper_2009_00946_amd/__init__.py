"""FEWHA tomography hot path for AMD MI355X (gfx950).

``fewha.Plan`` binds the HIP library (``libfewha.so``, C ABI in ``include/fewha.h``) to torch
device memory; ``synth`` draws the seeded synthetic inputs; ``configs/`` holds the AO
configurations.
"""

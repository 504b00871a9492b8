"""MI355X-native stochastic multiscale FEM upscaling (hot path).

The compute path is ``libstomsfem.so`` (hand-written HIP for gfx950 behind a
C ABI, see ``include/stomsfem.h``); :mod:`.stomsfem` is a thin ctypes binding
with the same entry-point names.  PyTorch is used only for device memory and
streams.
"""

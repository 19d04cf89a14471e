"""MI355X-native tent-pitched space-time Trefftz-DG (first-order acoustic wave
system).  The solver lives in libtdg.so (C++ host code and gfx950 HIP kernels,
C-ABI in include/tdg.h); ``tdg`` is its ctypes binding."""

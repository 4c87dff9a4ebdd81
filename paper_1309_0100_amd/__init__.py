"""MI355X-native implementation of the FREDEC multifrequency periodogram hot
path (Baluev, arXiv:1309.0100): a C-ABI HIP library (libfredec.so, built from
csrc/) and a thin ctypes binding (fredec.py).  Importing this package loads
nothing; the binding loads the library on first use."""

"""MI355X-native buffer update of the arbitrary-positioned SPH in-/outlet buffer
(arXiv 2406.16786).  The product is ``libsphbuf.so`` (C ABI in ``include/sphbuf.h``);
``sphbuf`` is its ctypes binding and ``domain`` a small torch-side holder of
particle arrays and a library context."""

"""MI355X fragment solver for periodic LNO-CCSD(T): closed-shell DF-CCSD and
(T) on one fragment's active space, as a HIP library with a C ABI
(include/lnocc.h) and this thin ctypes binding."""

"""FP64 CPU oracle of the FEWHA hot path (test infrastructure only).

Only the test suite, the smoke check and the CPU-baseline leg of the benchmark may import
this package; the product library never does.  ``Oracle(cfg)`` wraps the plain C
implementation in ``fewha_oracle.c`` through ctypes; the configuration dictionary (the
JSON under ``paper_2009_00946_amd/configs``) is parsed here, independently of the
library's own binding.
"""
from .oracle import Oracle, build, db3, get_threads, lib_path, set_threads  # noqa: F401

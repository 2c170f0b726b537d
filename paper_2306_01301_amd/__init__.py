"""MI355X-native kernel-style N-turn nonholonomic planner (arXiv 2306.01301).

The compute path is the HIP library ``libnhp.so`` (built from ``csrc/``) behind
the C ABI declared in ``include/nhp.h``; ``planner`` is its Python binding.
``scenes`` draws seeded synthetic inputs.  Importing this package loads
nothing; ``planner`` loads the library on first use and raises if it is
missing.
"""

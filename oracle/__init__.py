"""Reference implementation of the quasi-orthogonal method (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product path (the HIP library and
its Python binding) never imports, loads or calls anything in it.
"""
from .oracle import *  # noqa: F401,F403

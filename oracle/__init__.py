"""CPU oracle of the bit-box particle compressor -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product path never does.
"""
from .oracle import Oracle, OracleError, default  # noqa: F401

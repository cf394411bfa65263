"""CPU oracle of the complex Ozaki-II scheme (arXiv 2512.08321).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import anything from this
package.  The GPU library never imports, links or calls it, and the two share
no code: only the seeded input generators (``workloads.py``) serve both.

* ``oracle.reference`` - pure-Python exact reference (tiny shapes), the
  readable statement of the method.
* ``oracle.core``      - the same computation in C (``core.c``) for larger
  shapes and sampled entries, plus the double-double complex GEMM used as the
  accuracy yardstick.  Pinned against ``reference`` and against mathematical
  facts by the ``-m "not gpu"`` tests.

Parity pins: every function here is pinned by a test in
``tests/test_oracle_*.py``; none is "parity unpinned".
"""
from . import reference  # noqa: F401

"""CPU oracle for the km1 label-propagation refinement core.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The HIP library
and its Python binding share no code with it and never import it.
"""
from . import oracle  # noqa: F401

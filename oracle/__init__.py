"""CPU oracle for the overlapped RBF-FD differentiation-matrix build.

TEST INFRASTRUCTURE ONLY.  Imported by ``tests/``, by
``__graft_entry__.smoke()`` and by the CPU-baseline leg of ``bench.py``;
never by the product package ``paper_1606_03135_amd``, and it imports
nothing from it.  See ``oracle/orbf_oracle.c`` for the passages of the paper
each routine follows.
"""
from .oracle import *  # noqa: F401,F403

"""Exact CPU oracle for the m-double matrix product by error-free summation.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU leg of ``bench.py`` (its ``cpu_baseline`` and the error check of
sampled GPU outputs, after all GPU work) may import, call, link or execute
anything under ``oracle/``.  The product path (the HIP library and its Python
binding) never does, and shares no code with it.

Modules:

* ``oracle.exact``   plain Python with exact integers and ``fractions``: the
  exact product, the method's own integer steps (exponent alignment, split,
  diagonal sums, fold), round-to-nearest renormalisation, the nonoverlap
  predicate, the error report, the slice-count rule and exact gradients.
* ``oracle.mdarith`` ordinary m-double addition and multiplication built from
  published error-free transformations, with operation counters (checked
  against the paper's operation-count table) and quad-double arithmetic for
  the finite-difference gradient check.
* ``oracle.coracle`` ctypes loader for ``oracle/c/oracle.c``, a plain C port of
  the exact product and of the method's integer steps for large or sampled
  checks and for the timed CPU baseline.
"""

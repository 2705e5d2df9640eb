"""Seeded input generators shared by the oracle and the GPU path.

This package holds no decoding, mapping or channel arithmetic. It only:

* draws quasi-cyclic base matrices from a seed and reads/writes them as
  ``.qc`` text fixtures (``qc_base``),
* describes the workloads (code shape, modulation, Eb/N0 points, batch sizes,
  seeds) that the tests and the benchmark run (``workloads``),
* draws plain seeded random arrays used as test inputs (``rand``).

Both ``oracle/`` and ``paper_2203_11854_amd/`` consume what this package
produces; neither imports the other.
"""

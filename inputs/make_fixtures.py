"""Write every ``.qc`` fixture from its seed.

Run ``python -m inputs.make_fixtures`` from the repository root.  The output
is deterministic; ``tests/test_inputs.py`` checks that the committed files
equal a fresh draw.
"""
from __future__ import annotations

import os

from .qc_base import FIXTURE_DIR, fixture_path, write_qc
from .workloads import ALL_CODES


def main() -> None:
    os.makedirs(FIXTURE_DIR, exist_ok=True)
    for spec in ALL_CODES:
        qb = spec.draw()
        write_qc(fixture_path(spec.name), qb)
        nnz = int((qb.base[:spec.decoded_rows] >= 0).sum())
        print(f"{spec.name}: {qb.mb}x{qb.nb} Z={qb.Z} nnz(decoded rows)={nnz} "
              f"redraws={qb.meta['redraws']}")


if __name__ == "__main__":
    main()

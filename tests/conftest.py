import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


@pytest.fixture(scope="session")
def oracle_lib():
    import oracle
    oracle.build(force=False)
    return oracle


def load_golden_blocks(path):
    """Parse tests/golden/bc1_blocks.txt into [(c0, c1, idx, [[(n,d)x3]x4 cols]x4 rows)]."""
    from fractions import Fraction
    blocks = []
    cur = None
    with open(path) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            if line.startswith("block"):
                _, c0, c1, idx = line.split()
                cur = (int(c0, 16), int(c1, 16), int(idx, 16), [])
                blocks.append(cur)
                continue
            row = []
            for texel in line.split():
                row.append(tuple(Fraction(int(a), int(b)) for a, b in (p.split("/") for p in texel.split(","))))
            assert len(row) == 4
            cur[3].append(row)
    for b in blocks:
        assert len(b[3]) == 4
    return blocks

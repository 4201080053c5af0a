import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


def load_golden(name):
    """Parse a tests/golden fixture: 'key: values' lines, '#' comments."""
    out = {}
    with open(os.path.join(ROOT, "tests", "golden", name)) as fh:
        for line in fh:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            k, v = line.split(":", 1)
            vals = []
            for tok in v.split():
                if tok.startswith("0x"):
                    vals.append(int(tok, 16))
                else:
                    try:
                        vals.append(int(tok))
                    except ValueError:
                        vals.append(float(tok))
            out[k.strip()] = vals if len(vals) != 1 else vals[0]
    return out


@pytest.fixture
def golden():
    return load_golden

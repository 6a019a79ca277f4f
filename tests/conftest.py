import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: larger CPU cases")


@pytest.fixture(scope="session")
def oracle_mod():
    import oracle
    oracle.build(force=False)
    return oracle


@pytest.fixture(scope="session")
def datagen_mod():
    import datagen
    datagen.build(force=False)
    return datagen


def parse_golden(name):
    """Yield dict cases from a tests/golden/*.txt file (see the file headers)."""
    path = os.path.join(ROOT, "tests", "golden", name)
    cases = []
    with open(path) as f:
        for line in f:
            line = line.rstrip("\n")
            if not line.strip() or line.lstrip().startswith("#"):
                continue
            fields = [x.strip() for x in line.split("|")]
            while len(fields) < 6:
                fields.append("")
            toks = [bytes.fromhex(t) for t in fields[0].split(",")]
            cases.append({
                "line": line,
                "tokens": toks,
                "codes": fields[1].split() if fields[1] else [],
                "code_off": [int(x) for x in fields[2].split(",")],
                "status": int(fields[3]),
                "out_off": None if fields[4] == "-" else [int(x) for x in fields[4].split(",")],
                "bytes": None if fields[5] == "-" else bytes.fromhex(fields[5].replace(" ", "")),
            })
    return cases

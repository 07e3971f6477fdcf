import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library)")
    config.addinivalue_line("markers", "slow: larger CPU cases")


def parse_golden(path):
    """Parse tests/golden/paper_examples.txt into a list of cases."""
    cases = []
    cur = None
    with open(path) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            tok = line.split()
            if tok[0] == "case":
                cur = dict(name=tok[1], version=int(tok[2], 0), generator=int(tok[3], 0), recs=[], words=None)
            elif tok[0] == "rec":
                opnds, name = [], b""
                for t in tok[2:]:
                    if t.startswith("str="):
                        name = t[4:].encode()
                    else:
                        opnds.append(int(t, 0))
                cur["recs"].append((int(tok[1], 0), opnds, name))
            elif tok[0] == "words":
                cur["words"] = [int(t, 16) for t in tok[1:]]
            elif tok[0] == "end":
                cases.append(cur)
                cur = None
    return cases


@pytest.fixture(scope="session")
def golden_cases():
    return parse_golden(os.path.join(ROOT, "tests", "golden", "paper_examples.txt"))

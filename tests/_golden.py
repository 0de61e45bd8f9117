"""Reader for the small text fixtures under tests/golden/."""
import os

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def paper_constants():
    out = {}
    with open(os.path.join(GOLDEN, "paper_constants.txt")) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, val, _cite = line.split(None, 2)
            out[key] = float(val)
    return out

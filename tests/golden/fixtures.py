"""Reader for the small text fixtures next to this file."""
import os

HERE = os.path.dirname(os.path.abspath(__file__))


def read(name: str) -> dict:
    out = {}
    with open(os.path.join(HERE, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, *vals = line.split()
            out[key] = vals
    return out


def pairs(vals):
    return [tuple(int(t) for t in v.split(",")) for v in vals]

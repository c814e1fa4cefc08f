"""Reader for the paper-value fixtures in this folder (sections of numbers)."""
import os

HERE = os.path.dirname(os.path.abspath(__file__))


def load(name):
    out, cur = {}, None
    with open(os.path.join(HERE, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            if line.startswith("["):
                cur = line.strip("[]")
                out[cur] = []
                continue
            out[cur].append(line.split())
    return out

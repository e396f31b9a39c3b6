"""Reader for the paper's printed PCG iteration tables (Sec. 6.3)."""
import os

HERE = os.path.dirname(os.path.abspath(__file__))


def pcg_tables():
    out, cur = {}, None
    with open(os.path.join(HERE, "pcg_iterations_tables.txt")) as f:
        for line in f:
            line = line.split("#")[0].strip()
            if not line:
                continue
            if line.startswith("["):
                cur = line.strip("[]")
                out[cur] = {}
                continue
            v = line.split()
            out[cur][int(v[0])] = {p: float(x) for p, x in zip((1, 2, 3, 4), v[1:])}
    return out

"""The MHD Riemann problems of Sec. 3.1.4 (Table "Riemann Problem Initial
Conditions"), read from tests/golden/riemann_problems.txt."""
import math
import os

HERE = os.path.dirname(os.path.abspath(__file__))


def riemann_table():
    """[(name, {gamma, tmax, bx, left, right})]; left/right are sweep-frame
    primitives (rho, P, v_n, v_t1, v_t2, B_t1, B_t2)."""
    s4pi = math.sqrt(4 * math.pi)
    rows = []
    with open(os.path.join(HERE, "golden", "riemann_problems.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            tok = line.split()
            v = [eval(t, {"s4pi": s4pi}) for t in tok[1:]]  # noqa: S307 (fixture arithmetic)
            rows.append((tok[0], dict(gamma=v[0], tmax=v[1], bx=v[2], left=v[3:10], right=v[10:17])))
    return rows


def riemann_row(name):
    return dict(riemann_table())[name]

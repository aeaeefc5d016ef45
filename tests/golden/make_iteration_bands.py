"""Write tests/golden/iteration_bands.json: for each parity workload, the
range of PCG iteration counts that FP64 rounding order alone produces,
from the oracle only (oracle.msp_closed.band):

  * the oracle (MSP by elimination of T~, sequential sums) and eight runs
    of its rounding model (relative noise 4e-16 on L p and M r);
  * the same with every inner product and mean correctly rounded;
  * the MSP in closed form under both of the above.

Below mu = 0.5 the elimination is not accurate to FP64 rounding, so those
cases use the closed form alone (its own pin: tests/test_oracle_closed.py).
Tolerance 1e-8, x0 = 0, stop on the recursive residual (Sec. 4).

Run from the repository root:  python tests/golden/make_iteration_bands.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
sys.path.insert(0, os.path.dirname(HERE))

from cases import ELIM_MIN_MU, PCG_CASES, case, hub_case, plain_cg_case  # noqa: E402

TOL, MAXIT = 1e-8, 20000


def one(name, n, u, v, w, mu, b):
    from oracle import MSP, Graph, Hierarchy
    from oracle.msp_closed import band
    g = Graph(n, u, v, w)
    if mu is None:
        B = band(g, b, TOL, MAXIT)
    else:
        h = Hierarchy(g)
        if mu >= ELIM_MIN_MU:
            B = band(g, b, TOL, MAXIT, h=h, mu=mu, precond=MSP(h, mu))
        else:
            from oracle.msp_closed import closed_form
            B = band(g, b, TOL, MAXIT, precond=closed_form(h, mu))
            B["runs"] = [(t.replace("elim", "closed"), k) for t, k in B["runs"]]
    print(name, B["lo"], B["hi"], "oracle", B["oracle"], flush=True)
    return dict(lo=B["lo"], hi=B["hi"], oracle=B["oracle"], runs=B["runs"], mu=mu)


def main():
    out = {}
    for name in PCG_CASES:
        out[name] = one(name, *case(name))
    out["plain_cg_grid2d_32x20"] = one("plain_cg_grid2d_32x20", *plain_cg_case())
    out["hub_21267"] = one("hub_21267", *hub_case())
    with open(os.path.join(HERE, "iteration_bands.json"), "w") as f:
        json.dump(dict(tol=TOL, maxit=MAXIT, cases=out), f, indent=1)


if __name__ == "__main__":
    main()

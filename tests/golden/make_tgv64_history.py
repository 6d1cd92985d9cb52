"""Writes tgv64_history.txt: kinetic energy and dissipation of the 64^3
Taylor-Green vortex (Re 1600, Ma 0.1) every 50 of 1000 TVD-RK3 steps at a
fixed step (the CFL step of the initial state), computed by the oracle only.

    python tests/golden/make_tgv64_history.py
"""
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle.pyoracle import Oracle  # noqa: E402
from paper_2406_19494_amd import workloads as W  # noqa: E402


def main():
    case, P = W.tgv(64)
    o = Oracle(case)
    U = o.cons(P)
    dt = o.dt(U, case.cfl)
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tgv64_history.txt")
    rows = []
    t0 = time.time()
    for n in range(0, 1001):
        if n % 50 == 0:
            d = o.diag(U)
            rows.append((n, n * dt, d["ek"], d["eps"]))
            print(f"step {n} ek {d['ek']:.17e} eps {d['eps']:.17e} ({time.time() - t0:.0f} s)",
                  flush=True)
        if n < 1000:
            U = o.step(U, dt)
    with open(out, "w") as fh:
        fh.write("# 3D Taylor-Green vortex 64^3, Re 1600, Ma 0.1, Pr 0.71, power-law viscosity;\n")
        fh.write("# TVD-RK3 at the fixed step dt below (CFL 0.5 step of the initial state).\n")
        fh.write("# Volume-mean kinetic energy and mu |omega|^2 dissipation, from the oracle\n")
        fh.write("# (written by tests/golden/make_tgv64_history.py).\n")
        fh.write(f"dt {dt:.17e}\n")
        for n, t, ek, eps in rows:
            fh.write(f"{n} {t:.17e} {ek:.17e} {eps:.17e}\n")


if __name__ == "__main__":
    main()

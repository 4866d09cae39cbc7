"""Writes porous128_T400_gradient.json: reference derivatives of the porosity
objective on the full porous-channel workload (128^3 D3Q19, x/y periodic,
bounce-back walls outside z, F_x = 1e-5, u0 = 0.05, Smagorinsky C_S = 0.1,
tau0 = 0.6, porosity from the seeded smoothed noise, objective
J = c_s^2 (<rho>_{x=16} - <rho>_{x=112}) + <rho |u|^2 / 2> after T = 400
steps), at 16 cells drawn uniformly from the domain (seed 2506 + 5).

For each cell it stores
  - the central difference (J(phi + h e) - J(phi - h e)) / (2 h) of the FP64
    oracle, h = 1e-3 (at h = 1e-6 the rounding noise of J dominates), and
  - the oracle's forward-mode (dual-number) derivative dJ/dphi, exact up to
    rounding.

Only the oracle and the seeded input generators are used.  Runs for about
1.5 hours on 8 host cores; results are written after every cell, and a
rerun continues from the cells already stored.
Usage: python tests/golden/make_porous128_gradient.py
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as O  # noqa: E402
from paper_2506_21804_amd import inputs as I  # noqa: E402

OUT = os.path.join(HERE, "porous128_T400_gradient.json")
T = 400
H = 1e-3
NCELLS = 16


def _oracle(case, tangent=False):
    p = O.make_params(case.q, case.shape, periodic=case.periodic, tau0=case.tau0, cs_smag=case.cs_smag,
                      force=case.force)
    return O.Oracle(p, mask=case.mask, porosity=case.porosity, rho0=case.rho0, u0=case.u0, tangent=tangent)


def main():
    case = I.porous_channel(128)
    planes = tuple(int(v) for v in case.extra["planes"])
    cells = [int(c) for c in I.sample_cells(case.ncells, NCELLS, seed_offset=5)]
    res = {"source": __doc__.split("\n\n")[0].replace("\n", " "), "T": T, "h": H, "planes": list(planes),
           "shape": list(case.shape), "cells": cells, "fd": {}, "tangent": {}}
    if os.path.exists(OUT):
        old = json.load(open(OUT))
        if old.get("cells") == cells and old.get("T") == T and old.get("h") == H:
            res["fd"], res["tangent"] = old["fd"], old["tangent"]
    s = _oracle(case)
    s.step(T)
    res["J"] = s.objective(planes)[0]
    del s
    for kind in ("fd", "tangent"):
        for cell in cells:
            if str(cell) in res[kind]:
                continue
            t0 = time.time()
            if kind == "fd":
                Js = []
                for sgn in (1, -1):
                    c2 = I.porous_channel(128)
                    c2.porosity = case.porosity.copy()
                    c2.porosity[cell] += sgn * H
                    s = _oracle(c2)
                    s.step(T)
                    Js.append(s.objective(planes)[0])
                    del s
                val = (Js[0] - Js[1]) / (2 * H)
            else:
                s = _oracle(case, tangent=True)
                e = np.zeros(case.ncells)
                e[cell] = 1.0
                s.set_phi_tangent(e)
                s.step(T)
                val = s.objective(planes)[1]
                del s
            res[kind][str(cell)] = val
            with open(OUT, "w") as fh:
                json.dump(res, fh, indent=1)
            print(f"{kind} cell {cell}: {val:.12e} ({time.time() - t0:.0f} s)", flush=True)


if __name__ == "__main__":
    main()

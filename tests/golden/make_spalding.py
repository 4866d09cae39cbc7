"""Writes spalding_k041_E9.json: the Spalding law of Sec. 2.2.1 (Eq. (17)),
y+ = u+ + (exp(k u+) - 1 - k u+ - (k u+)^2/2 - (k u+)^3/6) / E, evaluated for
kappa = 0.41, E = 9 in 50-digit decimal arithmetic (exp summed as its own
power series here), i.e. the closed form itself, independent of any double-
precision implementation."""
import json
import os
from decimal import Decimal, getcontext

getcontext().prec = 50


def dexp(x: Decimal) -> Decimal:
    term, total, n = Decimal(1), Decimal(1), 0
    while True:
        n += 1
        term = term * x / n
        if abs(term) < Decimal(10) ** -45:
            return total + term
        total += term


def yplus(up: Decimal, kappa=Decimal("0.41"), E=Decimal(9)) -> Decimal:
    k = kappa * up
    return up + (dexp(k) - 1 - k - k * k / 2 - k * k * k / 6) / E


if __name__ == "__main__":
    ups = [1, 5, 10, 15, 20, 25]
    out = {
        "source": "Spalding law, Sec. 2.2.1 Eq. (17), kappa = 0.41, E = 9 (smooth wall); 50-digit decimal evaluation",
        "uplus": [float(u) for u in ups],
        "yplus": [float(yplus(Decimal(u))) for u in ups],
    }
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "spalding_k041_E9.json"), "w") as fh:
        json.dump(out, fh, indent=1)
    print(out)

"""Writes the closed-form pin fixtures in this folder with mpmath (40 digits).

boys_values.json : F_m(T) = 1F1(m+1/2; m+3/2; -T)/(2m+1)   (eq. boys_function)
ssss_values.json : (ss|ss) of normalised s Gaussians from the closed form of
                   eq. eri_base_case, N = (2a/pi)^{3/4}.

Nothing here calls the GPU library; run: python tests/golden/make_pins.py
"""
import json
import os

import mpmath as mp

HERE = os.path.dirname(os.path.abspath(__file__))
mp.mp.dps = 40


def boys(m, T):
    return mp.hyp1f1(m + mp.mpf(1) / 2, m + mp.mpf(3) / 2, -mp.mpf(T)) / (2 * m + 1)


def ssss(e, cen):
    e = [mp.mpf(x) for x in e]
    cen = [[mp.mpf(v) for v in c] for c in cen]
    a, b, c, d = e
    A, B, C, D = cen
    p, q = a + b, c + d
    P = [(a * A[k] + b * B[k]) / p for k in range(3)]
    Q = [(c * C[k] + d * D[k]) / q for k in range(3)]
    dAB = sum((A[k] - B[k]) ** 2 for k in range(3))
    dCD = sum((C[k] - D[k]) ** 2 for k in range(3))
    T = p * q / (p + q) * sum((P[k] - Q[k]) ** 2 for k in range(3))
    F0 = boys(0, T)
    N = 1
    for x in e:
        N *= (2 * x / mp.pi) ** mp.mpf("0.75")
    return N * mp.exp(-a * b / p * dAB - c * d / q * dCD) * 2 * mp.pi ** mp.mpf(2.5) / (p * q * mp.sqrt(p + q)) * F0


def main():
    vals = []
    for (m, T) in [(0, 1), (1, 1), (6, 5), (12, 30), (13, 100), (12, 1000), (0, 0.25),
                   (3, 7.5), (8, 0.01), (16, 45), (4, 2500)]:
        vals.append({"m": m, "T": T, "F": mp.nstr(boys(m, T), 25)})
    with open(os.path.join(HERE, "boys_values.json"), "w") as f:
        json.dump({"source": "mpmath hyp1f1, 40 digits (eq. boys_function)", "values": vals}, f, indent=1)
    z = [0, 0, 0]
    zz = [0, 0, 1.4]
    rows = [
        ("one centre, a=1", [1, 1, 1, 1], [z, z, z, z]),
        ("(sA sA|sB sB), a=1, R=1.4", [1, 1, 1, 1], [z, z, zz, zz]),
        ("(sA sB|sA sB), a=1, R=1.4", [1, 1, 1, 1], [z, zz, z, zz]),
        ("(sA sA'|sB sB'), a=0.5,2, R=1.4", [0.5, 2, 0.5, 2], [z, z, zz, zz]),
        ("four centres", [0.3, 1.7, 0.9, 12.0], [[0.1, -0.2, 0.3], [1.0, 0.5, -0.4], [-0.7, 0.2, 1.1], [0.4, -1.3, 0.0]]),
    ]
    out = []
    for lab, e, cen in rows:
        out.append({"label": lab, "exps": e, "centres": cen, "value": mp.nstr(ssss(e, cen), 25)})
    with open(os.path.join(HERE, "ssss_values.json"), "w") as f:
        json.dump({"source": "closed form of eq. eri_base_case in mpmath, normalised s primitives", "values": out}, f, indent=1)


if __name__ == "__main__":
    main()

"""Write two_level.json: the hand-derived two-level polarizability.

System: one occupied and one virtual orbital (X = 1, transition energy D = 1),
one product with vertex [[0, v], [v, 0]], v = 0.5, kernel f = 0.25, dipole
d = 1, occupation factor n = 2, broadening eps = 0.1.

From eq. response-mat, chi0(w) = n v^2 [1/(w - D + i eps) - 1/(w + D + i eps)]
= 2nDv^2 / (z^2 - D^2) with z = w + i eps.  Eq. sle then gives
X = chi0 d / (1 - chi0 f) = 2nDv^2 d / (z^2 - D^2 - 2nDv^2 f), and with the
sign reading alpha = -d X:  alpha(w) = -1 / ((w + 0.1 i)^2 - 1.25).
"""
import json
import os

D, v, f, d, n, eps = 1.0, 0.5, 0.25, 1.0, 2.0, 0.1


def alpha(w):
    z = complex(w, eps)
    s = 2 * n * D * v * v
    return -(d * d) * s / (z * z - D * D - s * f)


if __name__ == "__main__":
    ws = [0.0, 0.25, 0.5, 1.0, 1.118033988749895, 1.5, 2.0, -1.0]
    vals = [[w, float(f"{alpha(w).real:.12g}"), float(f"{alpha(w).imag:.12g}")] for w in ws]
    out = {
        "what": "alpha(w) of a two-level system, derived by hand from eqs. response-mat and sle",
        "params": {"D": D, "v": v, "f": f, "d": d, "n": n, "eps": eps},
        "closed_form": "alpha(w) = -1 / ((w + 0.1i)^2 - 1.25)",
        "values": vals,
        "columns": ["omega", "Re alpha", "Im alpha"],
    }
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "two_level.json"), "w") as fh:
        json.dump(out, fh, indent=1)
        fh.write("\n")

"""Write sampled entries of the oracle's chi0(w) z for a large synthetic system.

    python tests/golden/make_sampled_apply.py atoms200_orb9 [--seed 0]
           [--omegas 0.45,1.3] [--vectors 2] [--stride 41]

For each frequency the oracle (oracle.chi0_oracle.chi0_apply, matrix-free
sum over transitions) is applied to `vectors` seeded random complex vectors
(synth.seeded_complex, seeds 100, 101, ...) and to the x, y, z dipole drives.
Every `stride`-th entry of each output (and the last one) is stored with the
2-norm of the whole output, so a GPU test can compare the full-size operator
on these entries.  Output: tests/golden/sampled_apply_<workload>_s<seed>.json,
with the generator fingerprint.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import chi0_oracle as orc  # noqa: E402
from paper_1005_5340_amd import synth  # noqa: E402


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("workload")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--omegas", default="0.45,1.3")
    ap.add_argument("--vectors", type=int, default=2)
    ap.add_argument("--stride", type=int, default=41)
    a = ap.parse_args()
    s = synth.make_system(a.workload, a.seed)
    P = s.n_prod
    idx = sorted(set(range(0, P, a.stride)) | {P - 1})
    seeds = [100 + k for k in range(a.vectors)]
    Z = np.stack([synth.seeded_complex(P, sd) for sd in seeds] + [d.astype(complex) for d in s.drives("xyz")], 1)
    out_path = os.path.join(os.path.dirname(os.path.abspath(__file__)),
                            f"sampled_apply_{a.workload}_s{a.seed}.json")
    rec = {"what": "sampled entries of oracle chi0(omega) z (matrix-free sum over transitions)",
           "workload": a.workload, "seed": a.seed, "eps": s.eps, "fingerprint": synth.fingerprint(s),
           "vector_seeds": seeds, "drives_appended": "xyz", "index": idx, "omega": [],
           "out_re": [], "out_im": [], "out_norm": [], "seconds": []}
    for w in [float(x) for x in a.omegas.split(",")]:
        t = time.time()
        Y = orc.chi0_apply(s, w, Z)
        rec["omega"].append(w)
        rec["out_re"].append(Y[idx].real.T.tolist())
        rec["out_im"].append(Y[idx].imag.T.tolist())
        rec["out_norm"].append(np.linalg.norm(Y, axis=0).tolist())
        rec["seconds"].append(time.time() - t)
        with open(out_path + ".tmp", "w") as f:
            json.dump(rec, f)
        print(f"omega={w} done in {time.time() - t:.0f} s", flush=True)
    os.replace(out_path + ".tmp", out_path)


if __name__ == "__main__":
    main()

"""Write the oracle's polarizability for a whole synthetic workload to JSON.

    python tests/golden/make_reference.py atoms60_orb9 [--seed 0] [--omegas i,j,...] [--merge]

Calls only the FP64 oracle (oracle.chi0_oracle) on inputs from the seeded
generator; the file also stores the generator fingerprint so that a reader
on another machine can check that it holds the same inputs.  Output:
tests/golden/reference_<workload>_s<seed>.json with alpha[omega][k][i].
With --merge the frequencies are added to an existing file of the same
inputs (sorted by grid index); frequencies already stored are skipped.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import chi0_oracle as orc  # noqa: E402
from paper_1005_5340_amd import synth  # noqa: E402


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("workload")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--omegas", default="", help="comma-separated grid indices (default: all)")
    ap.add_argument("--merge", action="store_true", help="add to an existing reference of the same inputs")
    a = ap.parse_args()
    s = synth.make_system(a.workload, a.seed)
    idx = [int(i) for i in a.omegas.split(",")] if a.omegas else list(range(s.omegas.size))
    out_path = os.path.join(os.path.dirname(os.path.abspath(__file__)),
                            f"reference_{a.workload}_s{a.seed}.json")
    drives = s.drives()
    rec = {"what": "oracle polarizability alpha_ki(omega) = -d_k . X_i (dense chi0 + LU)",
           "workload": a.workload, "seed": a.seed, "drives": s.workload.drives,
           "eps": s.eps, "fingerprint": synth.fingerprint(s),
           "omega_index": [], "omega": [], "alpha_re": [], "alpha_im": [], "seconds": []}
    if a.merge and os.path.exists(out_path):
        old = json.load(open(out_path))
        if not synth.same_inputs(s, old["fingerprint"]) or old["drives"] != rec["drives"]:
            raise SystemExit(f"{out_path} holds other inputs; not merging")
        rec = old
        idx = [k for k in idx if k not in rec["omega_index"]]
    for k in idx:
        t = time.time()
        al = orc.polarizability(s, [s.omegas[k]], drives)[0]
        rec["omega_index"].append(k)
        rec["omega"].append(float(s.omegas[k]))
        rec["alpha_re"].append(al.real.tolist())
        rec["alpha_im"].append(al.imag.tolist())
        rec["seconds"].append(time.time() - t)
        order = sorted(range(len(rec["omega_index"])), key=lambda i: rec["omega_index"][i])
        for key in ("omega_index", "omega", "alpha_re", "alpha_im", "seconds"):
            rec[key] = [rec[key][i] for i in order]
        with open(out_path + ".tmp", "w") as f:
            json.dump(rec, f)
        print(f"omega[{k}]={s.omegas[k]:.5f} alpha={al[0,0]:.12e} {time.time()-t:.1f}s", flush=True)
    if idx:
        os.replace(out_path + ".tmp", out_path)


if __name__ == "__main__":
    main()

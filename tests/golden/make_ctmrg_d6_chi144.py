"""Write the oracle's outputs for the benchmark shape to ctmrg_d6_chi144_seed0.json.

Calls the CPU oracle only (oracle/ctmrg.py, Z2 form; the plain form runs the
first iterations beside it as a cross-check).  Input: the i.i.d. tensor of
paper_2410_11596_amd.inputs.iid_tensor(2, 6, 0) (d = 2, D = 6, N(0,1) entries
from seed 0, max-abs normalised), chi = 144, traced boundary, 12 iterations of
four directional moves.  The stored values are the gauge-invariant outputs the
GPU tests compare: kept sector sizes and kept spectra of every truncation,
delta after every iteration, the final corner spectra, the one- and two-site
RDMs, the Heisenberg energy, ln kappa and sampled entries of the one-site
environment.

Usage: python tests/golden/make_ctmrg_d6_chi144.py [--dense-check N]
(about 35 s per iteration of the Z2 form on 8 cores; the plain form's
iterations take several times longer).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import ctmrg  # noqa: E402
from paper_2410_11596_amd import inputs  # noqa: E402

OUT = os.path.join(HERE, "ctmrg_d6_chi144_seed0.json")
D, CHI, SEED, ITERS = 6, 144, 0, 12
N_EPS = 256


def eps_sample_indices(q):
    rng = np.random.default_rng(1234)
    return rng.integers(0, q ** 4, N_EPS)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--dense-check", type=int, default=2, help="iterations of the plain form run beside (0: none)")
    args = ap.parse_args()
    A = inputs.iid_tensor(2, D, SEED)
    t0 = time.time()
    z = ctmrg.Run(CHI, "z2", A=A)
    dn = ctmrg.Run(CHI, "dense", A=A) if args.dense_check > 0 else None
    for it in range(ITERS):
        z.step(1)
        msg = f"iteration {it + 1}: delta {z.deltas[-1]:.3e} kept {[r['kept'] for r in z.records[-4:]]}"
        if dn is not None and it < args.dense_check:
            dn.step(1)
            for rz, rd in zip(z.records[-4:], dn.records[-4:]):
                k = sum(rz["kept"])
                assert k == sum(rd["kept"])
                assert np.allclose(rz["spectrum"][:k], rd["spectrum"][:k], rtol=1e-10, atol=1e-14)
            assert abs(z.deltas[-1] - dn.deltas[-1]) < 1e-12
            msg += " (plain form agrees)"
        print(msg, f"{time.time() - t0:.0f} s", flush=True)
    h = ctmrg.heisenberg_bond()
    out = {
        "source": "oracle/ctmrg.py Z2 form (tests/golden/make_ctmrg_d6_chi144.py)",
        "input": "inputs.iid_tensor(2, 6, 0): d=2, D=6, i.i.d. N(0,1), seed 0, max-abs normalised",
        "chi": CHI, "iterations": ITERS, "tau": 1e-12,
        "dense_check_iterations": min(args.dense_check, ITERS),
        "records": [{"kept": [int(r["kept"][0]), int(r["kept"][1])],
                     "spectrum": [float(v) for v in r["spectrum"][: sum(r["kept"])]]} for r in z.records],
        "deltas": [float(v) for v in z.deltas],
        "corner_spectra": [[float(v) for v in s] for s in z._spec],
        "rho1": z.rho1().tolist(),
        "rho2_h": z.rho2("h").tolist(),
        "rho2_v": z.rho2("v").tolist(),
        "energy": z.energy(h),
        "log_kappa": z.log_kappa(),
    }
    eps = z.epsilon().reshape(-1)
    idx = eps_sample_indices(D * D)
    out["eps_index"] = [int(i) for i in idx]
    out["eps_value"] = [float(eps[i]) for i in idx]
    out["eps_max_abs"] = float(np.abs(eps).max())
    with open(OUT, "w") as f:
        json.dump(out, f, indent=0)
    print("wrote", OUT)


if __name__ == "__main__":
    main()

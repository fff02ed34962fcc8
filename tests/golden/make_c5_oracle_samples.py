"""Write tests/golden/c5_256cube_oracle_samples.json: sampled entries of the FP64 oracle's
gradient and Gauss-Newton Hessian-vector product on the 256^3 workload (band 64^3, Nt = 20;
inputs from tests/c5_inputs.py), for the GPU parity test at that size.

Only the oracle runs here (no library call).  The whole gradient and product are computed,
then per velocity component the script stores 384 uniformly drawn band entries and the 32
entries of largest |g| and of largest |Hv|, with the component's max |g|, max |L v|,
max |pi(b)| = max |g - L v| and max |Hv|, and the energy and 2-norms.  Takes a few minutes
and ~20 GB of host memory:
    python tests/golden/make_c5_oracle_samples.py
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))            # tests/ (c5_inputs)
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))   # repository root

import oracle as O  # noqa: E402
from c5_inputs import c5  # noqa: E402

OUT = os.path.join(HERE, "c5_256cube_oracle_samples.json")


def main():
    d = c5()
    prob = d["prob"]
    I0 = d["I0"].astype(np.float64)
    I1 = d["I1"].astype(np.float64)
    vh = d["vh"].astype(np.complex128)
    dv = d["dv"].astype(np.complex128)
    t = time.perf_counter()
    st = O.evaluate(vh, I0, I1, prob)
    print(f"evaluate {time.perf_counter() - t:.0f} s, E = {st.E!r}", flush=True)
    t = time.perf_counter()
    g = O.gradient(st)
    print(f"gradient {time.perf_counter() - t:.0f} s", flush=True)
    t = time.perf_counter()
    H = O.hessvec(st, dv)
    print(f"hessvec {time.perf_counter() - t:.0f} s", flush=True)
    Lv = O.L_hat(prob)[None] * O.project(vh, prob)
    rng = np.random.default_rng(20181)
    B = int(np.prod(prob.bshape))
    comps = []
    for c in range(3):
        gc, hc = g[c].ravel(), H[c].ravel()
        idx = set(rng.choice(B, 384, replace=False).tolist())
        idx |= set(np.argsort(-np.abs(gc))[:32].tolist())
        idx |= set(np.argsort(-np.abs(hc))[:32].tolist())
        idx = sorted(idx)
        comps.append({
            "index": idx,
            "g": [[float(gc[i].real), float(gc[i].imag)] for i in idx],
            "hv": [[float(hc[i].real), float(hc[i].imag)] for i in idx],
            "max_abs_g": float(np.abs(gc).max()),
            "max_abs_Lv": float(np.abs(Lv[c]).max()),
            "max_abs_pib": float(np.abs(gc - Lv[c].ravel()).max()),
            "max_abs_hv": float(np.abs(hc).max()),
        })
    rec = {
        "workload": "256^3 six-class shell phantoms (seeds 0 and 1), band 64^3, Nt = 20, "
                    "alpha = 1e-3, s = 2, sigma = 1; v~ = half of a random band velocity "
                    "scaled to 8 voxels; random admissible direction with max |dv~| = 1",
        "written_by": "tests/golden/make_c5_oracle_samples.py (FP64 oracle only)",
        "band_index_layout": "flat [kz][ky][kx] index of one velocity component",
        "E": float(st.E),
        "norm2_g": float(np.linalg.norm(g.ravel())),
        "norm2_Lv": float(np.linalg.norm(Lv.ravel())),
        "norm2_pib": float(np.linalg.norm((g - Lv).ravel())),
        "norm2_hv": float(np.linalg.norm(H.ravel())),
        "components": comps,
    }
    with open(OUT, "w") as f:
        json.dump(rec, f, separators=(",", ":"))
    print("wrote", OUT, os.path.getsize(OUT), "bytes", flush=True)


if __name__ == "__main__":
    main()

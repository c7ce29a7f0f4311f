"""Writes oracle_regression.json: the oracle's results on small seeded cases.

Calls only the oracle and the seeded input generators.  Run it again, and commit the
result together with the reason, only when the oracle's arithmetic changes on purpose.

  python tests/golden/make_oracle_regression.py
"""
import hashlib
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads  # noqa: E402


def digest(a) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def cases():
    pop = workloads.plain()
    p = oracle.params_of(pop)
    for name, prec in (("plain1k fp64 100 steps", oracle.FP64),
                       ("plain1k fp32 100 steps", oracle.FP32),
                       ("plain1k fp32k 100 steps", oracle.FP32_KAHAN)):
        r = oracle.run(p, pop.pos, pop.radius, pop.type, steps=100, precision=prec)
        yield name, {"interactions": int(r["interactions"]), "pos_sha256": digest(r["pos"]),
                     "pos_first": [float(v) for v in r["pos"][0]]}
    sph = workloads.spheroid(3000, seed=7, steps=0)
    ps = oracle.params_of(sph)
    r = oracle.run(ps, sph.pos, sph.radius, sph.type, steps=50)
    yield "spheroid3000 two types fp64 50 steps", {
        "interactions": int(r["interactions"]), "pos_sha256": digest(r["pos"])}
    vid, start, ids, occ = oracle.bin(ps, sph.pos)
    yield "spheroid3000 binning", {"vid_sha256": digest(vid), "start_sha256": digest(start),
                                   "ids_sha256": digest(ids), "occ_sha256": digest(occ)}
    g = oracle.run_growing(p, pop.pos, pop.radius, pop.type, steps=30, capacity=1500,
                           p_div=0.01, seed=5)
    yield "plain1k growing 30 steps", {"per_step_n": g["per_step_n"],
                                       "pos_sha256": digest(g["pos"])}


def main():
    out = {name: val for name, val in cases()}
    with open(os.path.join(HERE, "oracle_regression.json"), "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)
        f.write("\n")


if __name__ == "__main__":
    main()

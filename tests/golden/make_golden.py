"""Writes the stored expected values under tests/golden/ (calls only phantom/ and oracle/).

    python tests/golden/make_golden.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import fcm_ref  # noqa: E402
from phantom import PhantomParams, phantom, sha256  # noqa: E402

CASES = {
    "slice_200x200_seed1": PhantomParams(shape=(200, 200), seed=1),
    "volume_64x128x128_seed2": PhantomParams(shape=(64, 128, 128), seed=2),
    "slice_64x48_seed7_sigma3_bias20": PhantomParams(shape=(64, 48), seed=7, sigma=3.0, bias=0.2),
}


def main():
    hashes = {}
    for name, p in CASES.items():
        img, lab = phantom(p, with_labels=True)
        hashes[name] = {"image_sha256": sha256(img), "labels_sha256": sha256(lab),
                        "shape": list(p.shape), "seed": p.seed, "sigma": p.sigma, "bias": p.bias}
    with open(os.path.join(HERE, "phantom_hashes.json"), "w") as f:
        json.dump(hashes, f, indent=1, sort_keys=True)

    img = phantom(CASES["slice_200x200_seed1"])
    tr = fcm_ref.solve(img, 4, 2.0, 1e-5, 300)
    out = {"workload": "slice 200x200 seed 1, C=4, m=2, eps=1e-5, max_iter=300, linspace init",
           "T": tr.T, "status": tr.status,
           "v": [list(map(float, v)) for v in tr.v],
           "delta": [None] + [float(d) for d in tr.delta[1:]],
           "J": [float(j) for j in tr.J]}
    with open(os.path.join(HERE, "oracle_slice_200x200_c4_m2.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()

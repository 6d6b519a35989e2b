"""Write tests/golden/c2_image.json: SHA-256 digests of the oracle's full
wavelet matrix of the 2^28-symbol Zipf workload (uint32, sigma = 2^16,
Zipf(s=1.1) over a seed-permuted alphabet, seed 2), and of the input itself.

Only the oracle and the seeded generator run here (the input is drawn on the
host); nothing comes from the HIP library.  It takes about a minute and about
8 GiB of host memory:

    python tests/golden/make_c2_image.py
"""
import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.dirname(HERE))

import oracle  # noqa: E402
from imagewalk import array_digests  # noqa: E402
from paper_1610_03524_amd import inputs  # noqa: E402

N, SIGMA, SEED = 1 << 28, 1 << 16, 2


def main():
    t = time.time()
    S = inputs.c2_zipf(n=N, sigma=SIGMA, seed=SEED)
    s_digest = hashlib.sha256(S.tobytes()).hexdigest()
    t_gen = time.time() - t
    t = time.time()
    img = oracle.build_image(oracle.KIND_WM, S, SIGMA)
    t_build = time.time() - t
    rec = {"what": "oracle wavelet matrix of the Zipf workload: n=2^28 uint32, sigma=2^16, Zipf(s=1.1) "
                   "over a seed-permuted alphabet, seed 2 (host generator)",
           "n": N, "sigma": SIGMA, "seed": SEED, "input_sha256": s_digest,
           "image_bytes": int(img.size), "digests": array_digests(img),
           "made_by": "tests/golden/make_c2_image.py (oracle only)",
           "seconds": {"generate": round(t_gen, 1), "oracle_build": round(t_build, 1)}}
    with open(os.path.join(HERE, "c2_image.json"), "w") as f:
        json.dump(rec, f, indent=1)
    print(f"wrote c2_image.json: {len(rec['digests'])} digests, generate {t_gen:.1f} s, oracle {t_build:.1f} s")


if __name__ == "__main__":
    main()

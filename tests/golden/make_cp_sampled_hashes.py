"""Writes cp_sampled_hashes.txt: SHA-256 of sampled matmul_cp output ciphertexts computed by the
CPU oracle at the batched (L' = 512, hidden 1024, N = 8192) and served (N = 16384, four primes
+ two special, BERT-large and GPT-2-base shapes) geometries, whose full outputs the oracle takes
minutes to compute.  Calls only the oracle and the seeded input generators.

    python tests/golden/make_cp_sampled_hashes.py [case ...]

The GPU tests regenerate the same inputs (same seeds), run the library and compare the hash of
each sampled output's words ([2][level][N] uint64, little endian) with this file.
"""
import hashlib
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

OUT = os.path.join(HERE, "cp_sampled_hashes.txt")

# name: (ctx params (log_n, n_q, n_special, dnum), level, L, weight source, input seed, key seed, enc seed, sampled outputs)
CASES = {
    "c4_L500_D1024": ((13, 3, 1, 3), 2, 500, ("batch", 1024), 7, 907, 4007, (0, 77)),
    "c5_1024x4096_L200": ((14, 4, 2, 2), 3, 200, ("serve", 1, (1024, 4096)), 501, 6501, 7501, (3, 100)),
    "c5_4096x1024_L200": ((14, 4, 2, 2), 3, 200, ("serve", 2, (4096, 1024)), 502, 6502, 7502, (5,)),
    "c5_768x768_L100": ((14, 4, 2, 2), 3, 100, ("serve", 8, (768, 768)), 503, 6503, 7503, (0, 11)),
}
SCALE = 2.0 ** 40


def inputs(name):
    """(W, X) of a case, from the seeded generators"""
    from paper_2508_19525_amd import workloads as wl
    prm, level, L, src, xseed, kseed, eseed, outs = CASES[name]
    if src[0] == "batch":
        W = wl.batch_weights(src[1])
        X = wl.batch_activations(xseed, L, src[1])
    else:
        W = wl.serving_weights(src[1], src[2])
        X = np.random.default_rng(wl.seed_for(5, wl.ROLE_X) * 1000 + xseed).normal(0.0, 1.0, (L, src[2][0]))
    return W, X


def words_hash(words) -> str:
    return hashlib.sha256(np.ascontiguousarray(words, dtype=np.uint64).astype("<u8").tobytes()).hexdigest()


def oracle_outputs(name):
    import oracle
    from paper_2508_19525_amd import workloads as wl
    prm, level, L, src, xseed, kseed, eseed, outs = CASES[name]
    W, X = inputs(name)
    o = oracle.Context(*prm)
    lp = wl.lp_of(L)
    g = o.cp_geometry(lp, W.shape[0], W.shape[1])
    keys = oracle.Keys(o, kseed, o.cp_galois(lp, W.shape[0], W.shape[1]))
    xw = np.stack([keys.encrypt(o.encode_rns(o.pack_spatial(X, a), SCALE, level), level, eseed, a) for a in range(g["n_in"])])
    Y = keys.matmul_cp(xw, level, W, lp, outputs=list(outs))
    return {b: words_hash(Y[b]) for b in outs}


def load():
    """{(case, output): sha256} from the stored file"""
    table = {}
    for line in open(OUT):
        if line.strip() and not line.startswith("#"):
            name, b, h = line.split()
            table[(name, int(b))] = h
    return table


def main(names):
    table = load() if os.path.exists(OUT) else {}
    for name in names:
        t = time.time()
        for b, h in oracle_outputs(name).items():
            table[(name, b)] = h
        print(f"{name}: {time.time() - t:.0f} s", flush=True)
    with open(OUT, "w") as f:
        f.write("# SHA-256 of sampled oracle matmul_cp outputs (written by make_cp_sampled_hashes.py; case output sha256)\n")
        for (name, b), h in sorted(table.items()):
            f.write(f"{name} {b} {h}\n")


if __name__ == "__main__":
    main(sys.argv[1:] or list(CASES))

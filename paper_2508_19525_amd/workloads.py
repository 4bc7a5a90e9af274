"""Workload definitions and seeded synthetic inputs.

Shared by the tests, the benchmark and the smoke check.  Holds no CKKS arithmetic: only the
parameter sets and the seeded numpy generators of the plaintext tensors (activations,
weights, head matrices), with the shapes and value distributions of the paper's BERT-base /
BERT-large / GPT-2 workloads (synthetic stand-ins for the GLUE inputs and pretrained weights).

Seed rule: seed = 0xB1B0000 + 16 * config + role.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

ROLE_X, ROLE_W, ROLE_SK, ROLE_ENC, ROLE_KEYS, ROLE_MASK, ROLE_ARRIVALS = range(7)


def seed_for(config: int, role: int) -> int:
    return 0xB1B0000 + 16 * config + role


@dataclass(frozen=True)
class Params:
    log_n: int
    n_q: int
    n_special: int
    dnum: int
    log_scale: int

    @property
    def n(self):
        return 1 << self.log_n

    @property
    def scale(self):
        return float(2 ** self.log_scale)


# C1: plain matmul_cp, N=4096, 2 x 50-bit primes (+1 special, dnum 2), scale 2^30
C1 = dict(params=Params(12, 2, 1, 2, 30), L=32, d_in=32, d_out=32, x_dist="uniform", w_std=0.02)
# C2: BERT-base fused linear op, N=8192, 3 x 50-bit primes + 1 special (dnum 3), scale 2^40
C2 = dict(params=Params(13, 3, 1, 3, 40), L=128, d_in=768, d_out=768, x_dist="normal", w_std=0.02)
# C3: attention matmul_cc, N=16384, 4 x 50-bit primes + 2 special (dnum 2), scale 2^40
C3 = dict(params=Params(14, 4, 2, 2, 40), heads=12, L=128, d_head=64)
# C6: attention output -- Softmax x V_h (12 heads, 128 tokens, d_v = 64, V_h zero-padded to 128
# columns) and Concat(Att_h) W_O (768 x 768) on the dense diagonal packing; N=16384, 5 x 50-bit
# primes (three levels for the ct-ct product, one for the ct-pt product) + 2 special (dnum 3)
C6 = dict(params=Params(14, 5, 2, 3, 40), heads=12, L=128, d_v=64, d_out=768, w_std=0.02)
# C7: fused Q_h K_h^T from X -- X 128 x 768, W_Q and W_K 768 x 768 with columns reordered for the
# multi-head packing, then the ct-ct product with step 1 on the server; N=16384, 6 x 50-bit primes
# (one level for matmul_cp, four for the ct-ct product) + 2 special (dnum 3)
C7 = dict(params=Params(14, 6, 2, 3, 40), heads=12, L=128, d_model=768, d_head=64, w_std=0.02)


def activations(config: int, L: int, d: int, dist: str) -> np.ndarray:
    rng = np.random.default_rng(seed_for(config, ROLE_X))
    if dist == "uniform":
        return rng.uniform(-1.0, 1.0, (L, d))
    return rng.normal(0.0, 1.0, (L, d))


def weights(config: int, d_in: int, d_out: int, std: float) -> np.ndarray:
    rng = np.random.default_rng(seed_for(config, ROLE_W))
    return rng.normal(0.0, std, (d_in, d_out))


def pack_spatial(X: np.ndarray, slots: int, a: int) -> np.ndarray:
    """Spatial-first slot vector of ciphertext `a` for the L x D matrix X: element (i, j) sits in
    ciphertext j // c at slot i + L' (j mod c), L' = 2^ceil(log2 L), c = slots / L'; when the padded
    width D' = 2^ceil(log2 D) is below c the D' columns repeat c / D' times.  (A data layout,
    not CKKS arithmetic: the oracle and the library each implement their own.)"""
    L, D = X.shape
    lp = 1 << int(np.ceil(np.log2(L)))
    c = slots // lp
    dp = 1 << int(np.ceil(np.log2(D)))
    out = np.zeros(slots)
    for u in range(c):
        col = (u % dp) if dp < c else a * c + u
        if col < D:
            out[u * lp: u * lp + L] = X[:, col]
    return out


def unpack_spatial(vecs, L: int, D: int, slots: int) -> np.ndarray:
    lp = 1 << int(np.ceil(np.log2(L)))
    c = slots // lp
    out = np.zeros((L, D))
    for col in range(D):
        b, u = divmod(col, c)
        out[:, col] = vecs[b][u * lp: u * lp + L]
    return out


def head_groups(heads: int):
    """power-of-two head groups, largest first (12 -> [8, 4])"""
    out, h = [], heads
    while h > 0:
        g = 1
        while g * 2 <= h:
            g *= 2
        out.append(g)
        h -= g
    return out


def attention_weights(config: int, heads: int, L: int):
    """row-stochastic L x L matrices per head (softmax of seeded N(0, 1) logits): stand-ins for the
    attention weights the MPC softmax hands back"""
    rng = np.random.default_rng(seed_for(config, ROLE_X) + 1000)
    out = []
    for _ in range(heads):
        z = rng.normal(0.0, 1.0, (L, L))
        e = np.exp(z - z.max(axis=1, keepdims=True))
        out.append(e / e.sum(axis=1, keepdims=True))
    return out


def head_values(config: int, heads: int, L: int, d_v: int):
    rng = np.random.default_rng(seed_for(config, ROLE_X) + 2000)
    return [rng.normal(0.0, 1.0, (L, d_v)) for _ in range(heads)]


def pack_mhp(mats, H: int, L: int, d: int, a: int, operand: str, slots: int) -> np.ndarray:
    """Multi-head packing of operand ciphertext `a` of one head group (client side, before
    encryption): slot i + L'(h + H kappa) holds A_h{i, a c + kappa} for operand "A" and the
    row-pre-rotated B_h{a c + kappa, (i + kappa) mod L'} for operand "Bp" (B_h = mats[h], d rows and
    up to L' columns, the rest zero), with L' = 2^ceil(log2 L) and c = slots / (L' H)."""
    lp = 1 << int(np.ceil(np.log2(L)))
    c = slots // (lp * H)
    v = np.zeros(slots)
    i = np.arange(lp)
    for h in range(H):
        for kap in range(c):
            k = a * c + kap
            if k >= d:
                continue
            base = lp * (h + H * kap)
            if operand == "A":
                col = np.zeros(lp)
                col[:L] = mats[h][:, k]
                v[base: base + lp] = col
            else:
                j = (i + kap) % lp
                row = np.zeros(lp)
                row[:mats[h].shape[1]] = mats[h][k, :]
                v[base: base + lp] = row[j]
    return v


def unpack_diag(vecs, H: int, L: int, slots: int, g0: int = 0):
    """C_h (L x L) for each head of a group from its diagonal-packed output vectors: output g,
    slot i + L'(h + H kappa) holds C_h{i, (i + g c + kappa) mod L'}."""
    lp = 1 << int(np.ceil(np.log2(L)))
    c = slots // (lp * H)
    C = [np.zeros((lp, lp)) for _ in range(H)]
    i = np.arange(lp)
    for g, v in enumerate(vecs):
        for h in range(H):
            for kap in range(c):
                D = (g0 + g) * c + kap
                C[h][i, (i + D) % lp] = v[lp * (h + H * kap) + i]
    return [m[:L, :L] for m in C]


def dense_diag_layout(heads: int, L: int, d_v: int, slots: int):
    """Where the dense diagonal packing (the Softmax x V_h outputs, head groups concatenated)
    puts Att_h{i, j}: arrays (ct, slot, head, row, col) over every slot that holds an element.
    Output o of a group of H heads (c = slots / (L' H)) holds at slot i + L'(h + H kappa) the
    element (i, (i + o c + kappa) mod d_v') of head h, d_v' = 2^ceil(log2 d_v)."""
    lp = 1 << int(np.ceil(np.log2(L)))
    dvp = 1 << int(np.ceil(np.log2(d_v)))
    cts, sl, hs, rs, cs = [], [], [], [], []
    a, h0 = 0, 0
    i = np.arange(L)
    for H in head_groups(heads):
        c = slots // (lp * H)
        for o in range(dvp // c):
            for h in range(H):
                for kap in range(c):
                    col = (i + o * c + kap) % dvp
                    keep = col < d_v
                    n_k = int(keep.sum())
                    cts.append(np.full(n_k, a))
                    sl.append(i[keep] + lp * (h + H * kap))
                    hs.append(np.full(n_k, h0 + h))
                    rs.append(i[keep])
                    cs.append(col[keep])
            a += 1
        h0 += H
    return tuple(np.concatenate(x) for x in (cts, sl, hs, rs, cs))


# C4: 64 independent matmul_cp instances, lengths uniform in {16..512}, hidden 768 or 1024,
# one weight matrix per hidden size, N=8192, 3 primes (+1 special, dnum 3), scale 2^40
C4 = dict(params=Params(13, 3, 1, 3, 40), n_inst=64, L_lo=16, L_hi=512, hidden=(768, 1024), w_std=0.02)


def batch_instances(n_inst: int = 64, L_lo: int = 16, L_hi: int = 512, hidden=(768, 1024), config: int = 4):
    """[(L_i, D_i)] for the batched workload, seeded"""
    rng = np.random.default_rng(seed_for(config, ROLE_X))
    Ls = rng.integers(L_lo, L_hi + 1, n_inst)
    Ds = rng.choice(np.array(hidden), n_inst)
    return [(int(L), int(D)) for L, D in zip(Ls, Ds)]


def batch_activations(i: int, L: int, D: int, config: int = 4) -> np.ndarray:
    rng = np.random.default_rng(seed_for(config, ROLE_X) * 1000 + i)
    return rng.normal(0.0, 1.0, (L, D))


def batch_weights(D: int, std: float = 0.02, config: int = 4) -> np.ndarray:
    rng = np.random.default_rng(seed_for(config, ROLE_W) * 10000 + D)
    return rng.normal(0.0, std, (D, D))


def lp_of(L: int) -> int:
    return 1 << int(np.ceil(np.log2(L)))


# C5: serving -- Poisson arrivals of mixed BERT-large-shaped and GPT-2-base-shaped linear ops,
# lengths 16..512, N=16384, 4 primes (+2 special, dnum 2), scale 2^40
C5 = dict(params=Params(14, 4, 2, 2, 40), rate=50.0, L_lo=16, L_hi=512,
          ops={"bert_large": [(1024, 1024), (1024, 4096), (4096, 1024)], "gpt2_base": [(768, 768), (768, 3072), (3072, 768)]})


def serving_requests(n_req: int, rate: float, ops: dict, L_lo: int = 16, L_hi: int = 512, n_clients: int = 4, config: int = 5):
    """[(arrival_s, weight_id, (d_in, d_out), L, client)] with exponential inter-arrival times;
    model chosen 50/50, op uniformly within the model"""
    rng = np.random.default_rng(seed_for(config, ROLE_ARRIVALS))
    names = sorted(ops)
    table = [(mi * 8 + oi, shape) for mi, m in enumerate(names) for oi, shape in enumerate(ops[m])]
    out, t = [], 0.0
    for _ in range(n_req):
        t += rng.exponential(1.0 / rate)
        m = int(rng.integers(0, len(names)))
        o = int(rng.integers(0, len(ops[names[m]])))
        wid = m * 8 + o
        shape = dict(table)[wid]
        out.append((t, wid, shape, int(rng.integers(L_lo, L_hi + 1)), int(rng.integers(0, n_clients))))
    return out


def serving_weights(wid: int, shape, std: float = 0.02, config: int = 5) -> np.ndarray:
    rng = np.random.default_rng(seed_for(config, ROLE_W) * 100 + wid)
    return rng.normal(0.0, std, shape)

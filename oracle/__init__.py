"""CPU oracle for the RNS-CKKS server-side path of BLB (arXiv 2508.19525).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no code with the
HIP library under ``paper_2508_19525_amd``; the two meet only through the seeded input
generators in ``paper_2508_19525_amd.workloads`` (which hold none of the method's
arithmetic).

The numerical work lives in ``blb_oracle.c`` (plain C, ``unsigned __int128`` and ``%``,
a textbook NTT for ring products, quad precision for encode/decode).  This module is a thin
ctypes wrapper that marshals numpy arrays.  All polynomials are in coefficient form,
limb-major ``[poly][limb][N]`` uint64 residues.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "blb_oracle.c")
_LIB_PATH = os.path.join(_HERE, "libblb_oracle.so")

_u64p = np.ctypeslib.ndpointer(dtype=np.uint64, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_u32p = np.ctypeslib.ndpointer(dtype=np.uint32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_u8p = np.ctypeslib.ndpointer(dtype=np.uint8, flags="C_CONTIGUOUS")

TAG_SK, TAG_ENC_A, TAG_ENC_E, TAG_KEY_A, TAG_KEY_E, TAG_MASK = 1, 2, 3, 4, 5, 6
LIMB_INT = 0xFFFFFFFF


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain C + OpenMP + libquadmath)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-Wall", "-o", tmp, _SRC,
                               "-lquadmath", "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = C.CDLL(_LIB_PATH)
        vp = C.c_void_p
        sig = {
            "orc_primes": (C.c_int, [C.c_int, C.c_int, _u64p]),
            "orc_philox4x32_10": (None, [_u32p, _u32p, _u32p]),
            "orc_cdt_table": (None, [_u64p]),
            "orc_sample_uniform_poly": (None, [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint64, C.c_int, _u64p]),
            "orc_sample_ternary_poly": (None, [C.c_uint64, C.c_int, _i32p]),
            "orc_sample_gauss_poly": (None, [C.c_uint64, C.c_uint32, C.c_uint32, C.c_int, _i32p]),
            "orc_ctx_create": (vp, [C.c_int, C.c_int, C.c_int, C.c_int]),
            "orc_ctx_destroy": (None, [vp]),
            "orc_ctx_moduli": (None, [vp, _u64p]),
            "orc_ntt_forward": (None, [vp, C.c_int, _u64p]),
            "orc_ntt_inverse": (None, [vp, C.c_int, _u64p]),
            "orc_polymul": (None, [vp, C.c_int, _u64p, _u64p, _u64p]),
            "orc_automorphism": (None, [vp, C.c_int, _u64p, C.c_uint64, _u64p]),
            "orc_galois_elt": (C.c_uint64, [vp, C.c_int64]),
            "orc_encode": (C.c_int, [vp, _f64p, C.c_int64, C.c_double, _i64p]),
            "orc_encode_rns": (C.c_int, [vp, _f64p, C.c_int64, C.c_double, C.c_int, _u64p]),
            "orc_crt_centered": (None, [vp, _u64p, C.c_int, _f64p]),
            "orc_decode": (None, [vp, _u64p, C.c_int, C.c_double, C.c_int64, _f64p]),
            "orc_encode_cplx": (C.c_int, [vp, _f64p, _f64p, C.c_int64, C.c_double, _i64p]),
            "orc_encode_rns_cplx": (C.c_int, [vp, _f64p, _f64p, C.c_int64, C.c_double, C.c_int, _u64p]),
            "orc_decode_cplx": (None, [vp, _u64p, C.c_int, C.c_double, C.c_int64, _f64p, _f64p]),
            "orc_keygen": (vp, [vp, C.c_uint64, _u64p, C.c_int]),
            "orc_keys_destroy": (None, [vp]),
            "orc_keys_secret": (None, [vp, _i32p]),
            "orc_keys_swk": (C.c_int, [vp, C.c_uint64, _u64p]),
            "orc_encrypt": (None, [vp, _u64p, C.c_int, C.c_uint64, C.c_uint32, _u64p]),
            "orc_decrypt": (None, [vp, _u64p, C.c_int, C.c_int, _u64p]),
            "orc_rotate": (C.c_int, [vp, _u64p, C.c_int, C.c_int64, _u64p]),
            "orc_relinearize": (C.c_int, [vp, _u64p, C.c_int, _u64p]),
            "orc_rescale": (None, [vp, _u64p, C.c_int, C.c_int, _u64p]),
            "orc_cp_geometry": (None, [vp, C.c_int, C.c_int, C.c_int, _i32p]),
            "orc_pack_spatial": (None, [vp, _f64p, C.c_int, C.c_int, C.c_int, _f64p]),
            "orc_matmul_cp": (C.c_int, [vp, _u64p, C.c_int, _f64p, C.c_int, C.c_int, C.c_int, C.c_void_p, _u64p]),
            "orc_cp_galois": (C.c_int, [vp, C.c_int, C.c_int, C.c_int, _u64p]),
            "orc_mask_to_share": (None, [vp, _u64p, C.c_int, C.c_int, C.c_uint64, C.c_uint32, _u64p, _u64p]),
            "orc_add_share": (None, [vp, _u64p, C.c_int, _u64p, _u64p]),
            "orc_rotate_sum": (C.c_int, [vp, _u64p, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, _u64p]),
            "orc_num_threads": (C.c_int, []),
            "orc_set_threads": (C.c_int, [C.c_int]),
            "orc_cc_geometry": (None, [vp, C.c_int, C.c_int, C.c_int, _i32p]),
            "orc_rerandomize": (C.c_int, [vp, _u64p, C.c_int, C.c_uint64, C.c_uint32, C.c_int, _u64p]),
            "orc_matmul_cc": (C.c_int, [vp, _u64p, _u64p, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_void_p, _u64p]),
            "orc_cc_galois": (C.c_int, [vp, C.c_int, C.c_int, C.c_int, _u64p]),
            "orc_cc_sv_geometry": (None, [vp, C.c_int, C.c_int, C.c_int, _i32p]),
            "orc_mhp_weight": (C.c_int, [vp, _f64p, C.c_int, C.c_int, C.c_int, C.c_int, C.c_void_p]),
            "orc_matmul_cc_sv": (C.c_int, [vp, _u64p, _u64p, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_void_p,
                                           _u64p]),
            "orc_matmul_cp_diag": (C.c_int, [vp, _u64p, C.c_int, _f64p, C.c_int, C.c_int, C.c_int, C.c_int, C.c_void_p, _u64p]),
            "orc_matmul_cp_pack": (C.c_int, [vp, _u64p, C.c_int, _f64p, C.c_int, C.c_int, C.c_int, C.c_int, C.c_void_p, _u64p]),
            "orc_matmul_cp_diag_pack": (C.c_int, [vp, _u64p, C.c_int, _f64p, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_void_p,
                                                  _u64p]),
            "orc_ks_counts": (None, [_i64p, C.c_int]),
            "orc_ew_add": (None, [vp, _u64p, _u64p, C.c_int, _u64p]),
            "orc_ew_add_plain": (None, [vp, _u64p, _u64p, C.c_int, _u64p]),
            "orc_ew_mul_plain": (None, [vp, _u64p, _u64p, C.c_int, _u64p]),
            "orc_ew_mul_relin": (C.c_int, [vp, _u64p, _u64p, C.c_int, _u64p]),
            "orc_scalar_op": (C.c_int, [vp, _u64p, _u64p, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, _u64p]),
            "orc_cc_bsgs_split": (None, [vp, C.c_int, C.c_int, C.c_int, _i32p]),
            "orc_cc_galois_bsgs": (C.c_int, [vp, C.c_int, C.c_int, C.c_int, _u64p]),
            "orc_matmul_cc_sched": (C.c_int, [vp, _u64p, _u64p, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int,
                                              C.c_void_p, _u64p]),
            "orc_matmul_cc_sv_sched": (C.c_int, [vp, _u64p, _u64p, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int,
                                                 C.c_void_p, _u64p]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def ks_counts(reset: bool = False) -> tuple:
    """(rotations, relinearisations) key-switched since the last reset"""
    out = np.zeros(2, np.int64)
    lib().orc_ks_counts(out, 1 if reset else 0)
    return int(out[0]), int(out[1])


def set_threads(n: int) -> int:
    """thread count of the oracle's parallel loops from now on; returns the previous count"""
    return int(lib().orc_set_threads(n))


def num_threads() -> int:
    return int(lib().orc_num_threads())


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def primes(log_n: int, count: int) -> np.ndarray:
    out = np.zeros(count, np.uint64)
    if lib().orc_primes(log_n, count, out) != 0:
        raise ValueError("prime scan failed")
    return out


def philox4x32_10(ctr, key) -> np.ndarray:
    out = np.zeros(4, np.uint32)
    lib().orc_philox4x32_10(_c(ctr, np.uint32), _c(key, np.uint32), out)
    return out


def cdt_table() -> np.ndarray:
    out = np.zeros(20, np.uint64)
    lib().orc_cdt_table(out)
    return out


def sample_uniform(seed, limb, obj, tag, q, n) -> np.ndarray:
    out = np.zeros(n, np.uint64)
    lib().orc_sample_uniform_poly(seed, limb, obj, tag, int(q), n, out)
    return out


def sample_ternary(seed, n) -> np.ndarray:
    out = np.zeros(n, np.int32)
    lib().orc_sample_ternary_poly(seed, n, out)
    return out


def sample_gauss(seed, obj, tag, n) -> np.ndarray:
    out = np.zeros(n, np.int32)
    lib().orc_sample_gauss_poly(seed, obj, tag, n, out)
    return out


class Context:
    """Ring Z[X]/(X^N+1) with the RNS chain q_0..q_{n_q-1} and special primes p_0..p_{K-1}."""

    def __init__(self, log_n: int, n_q: int, n_special: int, dnum: int):
        self.log_n, self.n, self.n_q, self.n_special, self.dnum = log_n, 1 << log_n, n_q, n_special, dnum
        self.alpha = (n_q + dnum - 1) // dnum
        self._p = lib().orc_ctx_create(log_n, n_q, n_special, dnum)
        if not self._p:
            raise ValueError("bad parameters")
        m = np.zeros(n_q + n_special, np.uint64)
        lib().orc_ctx_moduli(self._p, m)
        self.moduli = m
        self.q = m[:n_q]
        self.p = m[n_q:]

    def __del__(self):
        if getattr(self, "_p", None):
            lib().orc_ctx_destroy(self._p)
            self._p = None

    @property
    def slots(self) -> int:
        return self.n // 2

    # ---- ring primitives (coefficient form) ----
    def ntt_forward(self, m, a):
        a = _c(a, np.uint64).copy()
        lib().orc_ntt_forward(self._p, m, a)
        return a

    def ntt_inverse(self, m, a):
        a = _c(a, np.uint64).copy()
        lib().orc_ntt_inverse(self._p, m, a)
        return a

    def polymul(self, m, a, b):
        r = np.zeros(self.n, np.uint64)
        lib().orc_polymul(self._p, m, _c(a, np.uint64), _c(b, np.uint64), r)
        return r

    def automorphism(self, m, a, g):
        r = np.zeros(self.n, np.uint64)
        lib().orc_automorphism(self._p, m, _c(a, np.uint64), int(g), r)
        return r

    def galois_elt(self, left_steps: int) -> int:
        return int(lib().orc_galois_elt(self._p, int(left_steps)))

    # ---- encode / decode ----
    def encode(self, m, delta: float) -> np.ndarray:
        m = _c(m, np.float64)
        out = np.zeros(self.n, np.int64)
        rc = lib().orc_encode(self._p, m, m.size, float(delta), out)
        if rc != 0:
            raise ValueError("encode overflow")
        return out

    def encode_rns(self, m, delta: float, level: int) -> np.ndarray:
        m = _c(m, np.float64)
        out = np.zeros((level + 1, self.n), np.uint64)
        rc = lib().orc_encode_rns(self._p, m, m.size, float(delta), level, out)
        if rc != 0:
            raise ValueError("encode overflow")
        return out

    def encode_cplx(self, m_re, m_im, delta: float) -> np.ndarray:
        """complex slots m_re + i m_im (equal lengths) -> signed integer coefficients"""
        m_re, m_im = _c(m_re, np.float64), _c(m_im, np.float64)
        assert m_re.size == m_im.size
        out = np.zeros(self.n, np.int64)
        if lib().orc_encode_cplx(self._p, m_re, m_im, m_re.size, float(delta), out) != 0:
            raise ValueError("encode overflow")
        return out

    def encode_rns_cplx(self, m_re, m_im, delta: float, level: int) -> np.ndarray:
        m_re, m_im = _c(m_re, np.float64), _c(m_im, np.float64)
        assert m_re.size == m_im.size
        out = np.zeros((level + 1, self.n), np.uint64)
        if lib().orc_encode_rns_cplx(self._p, m_re, m_im, m_re.size, float(delta), level, out) != 0:
            raise ValueError("encode overflow")
        return out

    def decode_cplx(self, poly, level: int, delta: float, n_vals: int | None = None):
        """(real parts, imaginary parts) of the slots"""
        n_vals = self.slots if n_vals is None else n_vals
        re = np.zeros(n_vals, np.float64)
        im = np.zeros(n_vals, np.float64)
        lib().orc_decode_cplx(self._p, _c(poly, np.uint64), level, float(delta), n_vals, re, im)
        return re, im

    def crt_centered(self, poly, level: int) -> np.ndarray:
        out = np.zeros(self.n, np.float64)
        lib().orc_crt_centered(self._p, _c(poly, np.uint64), level, out)
        return out

    def decode(self, poly, level: int, delta: float, n_vals: int | None = None) -> np.ndarray:
        n_vals = self.slots if n_vals is None else n_vals
        out = np.zeros(n_vals, np.float64)
        lib().orc_decode(self._p, _c(poly, np.uint64), level, float(delta), n_vals, out)
        return out

    def rescale(self, ct, level: int) -> np.ndarray:
        ct = _c(ct, np.uint64)
        n_poly = ct.size // ((level + 1) * self.n)
        out = np.zeros((n_poly, level, self.n), np.uint64)
        lib().orc_rescale(self._p, ct, level, n_poly, out)
        return out

    # ---- matmul_cp geometry / packing ----
    def cp_geometry(self, L, d_in, d_out) -> dict:
        g = np.zeros(8, np.int32)
        lib().orc_cp_geometry(self._p, L, d_in, d_out, g)
        return dict(zip(["Lp", "c", "c_eff", "c_out", "n_in", "n_out", "B", "G"], [int(v) for v in g]))

    def pack_spatial(self, X, a: int) -> np.ndarray:
        X = _c(X, np.float64)
        out = np.zeros(self.slots, np.float64)
        lib().orc_pack_spatial(self._p, X, X.shape[0], X.shape[1], a, out)
        return out

    def cp_galois(self, L, d_in, d_out) -> np.ndarray:
        out = np.zeros(64, np.uint64)
        k = lib().orc_cp_galois(self._p, L, d_in, d_out, out)
        return out[:k].copy()

    # ---- matmul_cc geometry ----
    def cc_geometry(self, H_g, L, d) -> dict:
        g = np.zeros(4, np.int32)
        lib().orc_cc_geometry(self._p, H_g, L, d, g)
        return dict(zip(["Lp", "c", "n_ct", "n_out"], [int(v) for v in g]))

    def cc_galois(self, H_g, L, d, schedule: int = 0) -> np.ndarray:
        """Galois elements one head group's matmul_cc uses (schedule 1: BSGS; duplicates removed)"""
        out = np.zeros(4096, np.uint64)
        f = lib().orc_cc_galois_bsgs if schedule else lib().orc_cc_galois
        k = f(self._p, H_g, L, d, out)
        return np.unique(out[:k])

    def cc_bsgs_split(self, H_g, L, d) -> dict:
        """BSGS split of step 2 (B baby x G giant = L') and of step 1 (b1 x g1 = c)"""
        g = np.zeros(4, np.int32)
        lib().orc_cc_bsgs_split(self._p, H_g, L, d, g)
        return dict(zip(["B", "G", "b1", "g1"], [int(v) for v in g]))

    def cc_sv_geometry(self, H_g, L, d_v) -> dict:
        """Softmax x V_h for one head group: L', c, operand cts (reduction d = L), dense outputs
        (0: unsupported), d_v' = 2^ceil(log2 d_v)"""
        g = np.zeros(5, np.int32)
        lib().orc_cc_sv_geometry(self._p, H_g, L, d_v, g)
        return dict(zip(["Lp", "c", "n_ct", "n_out", "dvp"], [int(v) for v in g]))

    def mhp_weight(self, W, n_heads: int, d_head: int, L: int) -> np.ndarray:
        """W (d_in x n_heads d_head) with its columns reordered so that matmul_cp's spatial-first
        output is the multi-head packing of the ct-ct operands (head groups concatenated)"""
        W = _c(W, np.float64)
        n_cols = lib().orc_mhp_weight(self._p, W, W.shape[0], n_heads, d_head, L, None)
        if n_cols < 0:
            raise ValueError("unsupported multi-head geometry")
        out = np.zeros((W.shape[0], n_cols), np.float64)
        lib().orc_mhp_weight(self._p, W, W.shape[0], n_heads, d_head, L, out.ctypes.data_as(C.c_void_p))
        return out

    def pack_mhp(self, mats, H_g, L, d, a, operand):
        """Multi-head packing of ciphertext a for one head group: operand 'A' puts A_h{i, a c + kappa}
        at slot i + L'(h + H_g kappa); operand 'Bp' puts B_h{a c + kappa, (i + kappa) mod L'} there
        (B_h = mats[h], d rows and at most L' columns, rows pre-rotated by kappa)."""
        g = self.cc_geometry(H_g, L, d)
        lp, cc = g["Lp"], g["c"]
        v = np.zeros(self.slots)
        for h in range(H_g):
            for kap in range(cc):
                k = a * cc + kap
                if k >= d:
                    continue
                base = lp * (h + H_g * kap)
                for i in range(lp):
                    if operand == "A":
                        v[base + i] = mats[h][i, k] if i < L else 0.0
                    else:
                        j = (i + kap) % lp
                        v[base + i] = mats[h][k, j] if j < mats[h].shape[1] else 0.0
        return v

    def add_share(self, ct, level: int, share) -> np.ndarray:
        """(c0 + share, c1) mod q_i: the server's step of the MPC-to-CKKS conversion"""
        out = np.zeros((2, level + 1, self.n), np.uint64)
        lib().orc_add_share(self._p, _c(ct, np.uint64), level, _c(share, np.uint64), out)
        return out

    def ew_add(self, a, b, level: int) -> np.ndarray:
        """ewadd_cc: a + b"""
        out = np.zeros((2, level + 1, self.n), np.uint64)
        lib().orc_ew_add(self._p, _c(a, np.uint64), _c(b, np.uint64), level, out)
        return out

    def ew_add_plain(self, a, pt, level: int) -> np.ndarray:
        """ewadd_cp: (c0 + pt, c1), pt coefficient form [level+1][N]"""
        out = np.zeros((2, level + 1, self.n), np.uint64)
        lib().orc_ew_add_plain(self._p, _c(a, np.uint64), _c(pt, np.uint64), level, out)
        return out

    def ew_mul_plain(self, a, pt, level: int) -> np.ndarray:
        """ewmul_cp: (c0 pt, c1 pt), pt coefficient form [level+1][N]"""
        out = np.zeros((2, level + 1, self.n), np.uint64)
        lib().orc_ew_mul_plain(self._p, _c(a, np.uint64), _c(pt, np.uint64), level, out)
        return out

    def mask_to_share(self, ct, level: int, target_level: int, seed: int, ct_id: int):
        masked = np.zeros((2, target_level + 1, self.n), np.uint64)
        share = np.zeros((target_level + 1, self.n), np.uint64)
        lib().orc_mask_to_share(self._p, _c(ct, np.uint64), level, target_level, seed, ct_id, masked, share)
        return masked, share


class Keys:
    """Secret key, relinearisation key and Galois keys (all host-side, coefficient form)."""

    def __init__(self, ctx: Context, seed: int, galois=()):
        self.ctx = ctx
        self.galois = [int(g) for g in galois]
        arr = np.array(self.galois if self.galois else [0], np.uint64)
        self._p = lib().orc_keygen(ctx._p, seed, arr, len(self.galois))

    def __del__(self):
        if getattr(self, "_p", None):
            lib().orc_keys_destroy(self._p)
            self._p = None

    @property
    def secret(self) -> np.ndarray:
        s = np.zeros(self.ctx.n, np.int32)
        lib().orc_keys_secret(self._p, s)
        return s

    def switching_key(self, key_id: int) -> np.ndarray:
        c = self.ctx
        out = np.zeros((c.dnum, 2, c.n_q + c.n_special, c.n), np.uint64)
        if lib().orc_keys_swk(self._p, key_id, out) != 0:
            raise KeyError(key_id)
        return out

    def encrypt(self, pt, level: int, seed: int, ct_id: int = 0) -> np.ndarray:
        out = np.zeros((2, level + 1, self.ctx.n), np.uint64)
        lib().orc_encrypt(self._p, _c(pt, np.uint64), level, seed, ct_id, out)
        return out

    def decrypt(self, ct, level: int) -> np.ndarray:
        ct = _c(ct, np.uint64)
        degree = ct.size // ((level + 1) * self.ctx.n) - 1
        out = np.zeros((level + 1, self.ctx.n), np.uint64)
        lib().orc_decrypt(self._p, ct, level, degree, out)
        return out

    def rotate(self, ct, level: int, steps: int) -> np.ndarray:
        out = np.zeros((2, level + 1, self.ctx.n), np.uint64)
        if lib().orc_rotate(self._p, _c(ct, np.uint64), level, int(steps), out) != 0:
            raise KeyError("missing Galois key")
        return out

    def relinearize(self, ct3, level: int) -> np.ndarray:
        out = np.zeros((2, level + 1, self.ctx.n), np.uint64)
        if lib().orc_relinearize(self._p, _c(ct3, np.uint64), level, out) != 0:
            raise KeyError("missing relinearisation key")
        return out

    def rotate_sum(self, ct, level: int, block: int, n_blocks: int, direction: int = 0, mask=None) -> np.ndarray:
        """rotate-and-sum over n_blocks blocks of `block` slots: summation (direction 0, with the
        first-block mask unless mask=False) or broadcast (direction 1, never masked)"""
        if mask is None:
            mask = direction == 0
        lv = level - 1 if mask else level
        out = np.zeros((2, lv + 1, self.ctx.n), np.uint64)
        rc = lib().orc_rotate_sum(self._p, _c(ct, np.uint64), level, block, n_blocks, direction, 1 if mask else 0, out)
        if rc == -1:
            raise KeyError("missing Galois key")
        if rc != 0:
            raise ValueError("rotate_sum: bad arguments")
        return out

    def ew_mul_relin(self, a, b, level: int) -> np.ndarray:
        """ewmul_cc: the tensor of a and b, relinearised"""
        out = np.zeros((2, level + 1, self.ctx.n), np.uint64)
        if lib().orc_ew_mul_relin(self._p, _c(a, np.uint64), _c(b, np.uint64), level, out) != 0:
            raise KeyError("missing relinearisation key")
        return out

    def scalar_op(self, a, s, level: int, block: int, n_blocks: int, op: int, from_sum: bool = False) -> np.ndarray:
        """sadd (op 0) / smul (op 1) of a with the broadcast of s's first block, or (from_sum) with the
        unmasked rotate-and-sum of s"""
        out = np.zeros((2, level + 1, self.ctx.n), np.uint64)
        rc = lib().orc_scalar_op(self._p, _c(a, np.uint64), _c(s, np.uint64), level, block, n_blocks, op, 1 if from_sum else 0, out)
        if rc != 0:
            raise ValueError(f"scalar_op failed ({rc})")
        return out

    def rerandomize(self, ct, level: int, seed: int, ct_id: int, flood_bits: int) -> np.ndarray:
        """ct + Enc_pk(0) with a flooding term uniform in [-2^F, 2^F] (coefficient form)"""
        out = np.zeros((2, level + 1, self.ctx.n), np.uint64)
        if lib().orc_rerandomize(self._p, _c(ct, np.uint64), level, seed, ct_id, flood_bits, out) != 0:
            raise ValueError("rerandomize: bad arguments")
        return out

    def matmul_cc(self, A_cts, Bp_cts, level: int, H_g: int, L: int, d: int, outputs=None, b_prerotated=True,
                  schedule: int = 0) -> np.ndarray:
        """One head group; A_cts / Bp_cts: [n_ct][2][level+1][N]; returns [n_out][2][level-2][N]
        (B pre-rotated by the client) or [n_out][2][level-3][N] (step 1 run homomorphically)."""
        c = self.ctx
        g = c.cc_geometry(H_g, L, d)
        O = np.zeros((g["n_out"], 2, level - (2 if b_prerotated else 3), c.n), np.uint64)
        mask = None
        if outputs is not None:
            m = np.zeros(g["n_out"], np.uint8)
            m[list(outputs)] = 1
            mask = m.ctypes.data_as(C.c_void_p)
        rc = lib().orc_matmul_cc_sched(self._p, _c(A_cts, np.uint64), _c(Bp_cts, np.uint64), g["n_ct"], level, H_g, L, d,
                                       1 if b_prerotated else 0, schedule, mask, O)
        if rc != 0:
            raise ValueError(f"matmul_cc failed ({rc})")
        return O

    def matmul_cc_sv(self, A_cts, B_cts, level: int, H_g: int, L: int, d_v: int, outputs=None, b_prerotated=True,
                     schedule: int = 0) -> np.ndarray:
        """Softmax x V_h for one head group (A = attention weights, L x L; B = V_h, L x d_v, zero-padded
        to L' columns); returns the dense diagonal-packed outputs [d_v'/c][2][level-2 or level-3][N]"""
        c = self.ctx
        g = c.cc_sv_geometry(H_g, L, d_v)
        if g["n_out"] < 1:
            raise ValueError("unsupported Softmax x V geometry")
        O = np.zeros((g["n_out"], 2, level - (2 if b_prerotated else 3), c.n), np.uint64)
        mask = None
        if outputs is not None:
            m = np.zeros(g["n_out"], np.uint8)
            m[list(outputs)] = 1
            mask = m.ctypes.data_as(C.c_void_p)
        rc = lib().orc_matmul_cc_sv_sched(self._p, _c(A_cts, np.uint64), _c(B_cts, np.uint64), g["n_ct"], level, H_g, L, d_v,
                                          1 if b_prerotated else 0, schedule, mask, O)
        if rc != 0:
            raise ValueError(f"matmul_cc_sv failed ({rc})")
        return O

    def matmul_cp_diag(self, X_cts, level: int, W, L: int, n_heads: int, d_v: int, outputs=None, cplx: bool = False) -> np.ndarray:
        """Concat(Att_h) W from the dense diagonal-packed Att_h (head groups concatenated); W is
        (n_heads d_v) x d_out; returns the spatial-first outputs [n_out][2][level][N] (with cplx,
        ceil(n_out / 2) outputs, output b holding blocks 2b and 2b + 1 in the real and imaginary
        parts)"""
        c = self.ctx
        W = _c(W, np.float64)
        d_out = W.shape[1]
        assert W.shape[0] == n_heads * d_v
        dvp = 1 << int(np.ceil(np.log2(d_v)))
        g = c.cp_geometry(L, n_heads * dvp, d_out)
        n_y = (g["n_out"] + 1) // 2 if cplx else g["n_out"]
        Y = np.zeros((n_y, 2, level, c.n), np.uint64)
        mask = None
        if outputs is not None:
            m = np.zeros(n_y, np.uint8)
            m[list(outputs)] = 1
            mask = m.ctypes.data_as(C.c_void_p)
        rc = lib().orc_matmul_cp_diag_pack(self._p, _c(X_cts, np.uint64), level, W, L, n_heads, d_v, d_out, 1 if cplx else 0, mask, Y)
        if rc != 0:
            raise ValueError(f"matmul_cp_diag failed ({rc})")
        return Y

    def matmul_cp(self, X_cts, level: int, W, L: int, outputs=None, cplx: bool = False) -> np.ndarray:
        """X W in the spatial-first packing; with cplx the complex-slot output packing
        (ceil(n_out / 2) outputs, output b holding blocks 2b and 2b + 1 in the real and
        imaginary parts of its slots)"""
        c = self.ctx
        W = _c(W, np.float64)
        d_in, d_out = W.shape
        g = c.cp_geometry(L, d_in, d_out)
        n_y = (g["n_out"] + 1) // 2 if cplx else g["n_out"]
        Y = np.zeros((n_y, 2, level, c.n), np.uint64)
        mask = None
        if outputs is not None:
            m = np.zeros(n_y, np.uint8)
            m[list(outputs)] = 1
            mask = m.ctypes.data_as(C.c_void_p)
        rc = lib().orc_matmul_cp_pack(self._p, _c(X_cts, np.uint64), level, W, L, d_in, d_out, 1 if cplx else 0, mask, Y)
        if rc != 0:
            raise KeyError("missing Galois key")
        return Y

"""Python face of the CPU oracle (``rdl_oracle.c``).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark call this module; the product path never does.  It loads
``liboracle.so`` built from ``rdl_oracle.c`` and ``rdl_ent_oracle.c`` (the
entropy code of the enhancement layer) by :func:`build` (plain gcc, no
fast-math, no FMA contraction) and wraps each stage so that it takes and
returns numpy arrays.  Nothing here does any of the method's arithmetic.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rdl_oracle.c")
_SRCS = [_SRC, os.path.join(_HERE, "rdl_ent_oracle.c"), os.path.join(_HERE, "rdl_jpeg_oracle.c")]
_LIB = os.path.join(_HERE, "liboracle.so")
CFLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared"]

_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle with gcc into ``oracle/liboracle.so``."""
    if force or not os.path.exists(_LIB) or any(os.path.getmtime(_LIB) < os.path.getmtime(f) for f in _SRCS):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, *_SRCS, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(_LIB)
        vp, i64, i32 = C.c_void_p, C.c_int64, C.c_int32
        L.oracle_tables.argtypes = [vp] * 5
        L.oracle_keystat.argtypes = [vp, i64, vp, vp]
        L.oracle_key_params.argtypes = [i64, i64, vp, vp, vp]
        L.oracle_tmo.argtypes = [vp, C.c_int, C.c_int, i32, C.c_float, i64, vp]
        L.oracle_quant_table.argtypes = [C.c_int, C.c_int, vp]
        L.oracle_fdct_block.argtypes = [vp, vp]
        L.oracle_idct_block.argtypes = [vp, vp]
        L.oracle_quantise.argtypes = [i32, i32]
        L.oracle_quantise.restype = i32
        L.oracle_base_layer.argtypes = [vp, C.c_int, C.c_int, C.c_int, vp, vp]
        L.oracle_gf.argtypes = [vp, C.c_int, C.c_int, vp]
        L.oracle_base_decode.argtypes = [vp, C.c_int, C.c_int, C.c_int, vp]
        L.oracle_base_decode.restype = C.c_int
        L.oracle_sums.argtypes = [vp, vp, i64, vp]
        L.oracle_solve.argtypes = [vp, vp, vp, vp]
        L.oracle_mstar.argtypes = [i32, i32, i32]
        L.oracle_mstar.restype = i32
        L.oracle_resid.argtypes = [vp, vp, i64, vp, vp, vp]
        L.oracle_encode_enh.argtypes = [vp, C.c_int, C.c_int, C.c_int, vp, vp, vp, vp, vp, vp, vp]
        L.oracle_encode_enh.restype = C.c_int
        L.oracle_decode_enh.argtypes = [vp, vp, vp, vp, C.c_int, C.c_int, vp]
        L.oracle_decode_enh.restype = C.c_int
        L.oracle_encode_mode.argtypes = [vp, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, vp, vp, vp, vp, vp]
        L.oracle_encode_mode.restype = C.c_int
        L.oracle_decode_mode.argtypes = [vp, vp, vp, vp, C.c_int, C.c_int, C.c_int, vp]
        L.oracle_decode_mode.restype = C.c_int
        L.oracle_resid_hist.argtypes = [vp, i64, vp]
        L.oracle_mlp_estimate.argtypes = [vp, vp, vp, C.c_int, C.c_int, i32, vp, vp]
        L.oracle_mlp_estimate.restype = C.c_int
        L.oracle_log2q16.argtypes = [i64]
        L.oracle_log2q16.restype = i64
        L.oracle_hist_cost.argtypes = [vp, C.c_int]
        L.oracle_hist_cost.restype = i64
        L.oracle_cross_cost.argtypes = [vp, vp, i64, C.c_int]
        L.oracle_cross_cost.restype = i64
        L.oracle_encode_learned.argtypes = [vp, C.c_int, C.c_int, C.c_int, vp, vp, vp, vp, vp, vp, vp, vp]
        L.oracle_encode_learned.restype = C.c_int
        L.oracle_decode_learned.argtypes = [vp, vp, vp, vp, i32, vp, vp, C.c_int, C.c_int, vp]
        L.oracle_decode_learned.restype = C.c_int
        L.oracle_jpeg_huff_table.argtypes = [vp, vp, vp]
        L.oracle_jpeg_huff_table.restype = C.c_int
        L.oracle_jpeg_write.argtypes = [vp, C.c_int, C.c_int, C.c_int, vp, i64]
        L.oracle_jpeg_write.restype = i64
        L.oracle_ent_freqs.argtypes = [vp, C.c_int, vp]
        L.oracle_ent_freqs.restype = C.c_int
        L.oracle_ent_bound.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int]
        L.oracle_ent_bound.restype = i64
        L.oracle_ent_encode.argtypes = [vp, vp, C.c_int, C.c_int, C.c_int, C.c_int, vp, i64]
        L.oracle_ent_encode.restype = i64
        L.oracle_ent_decode.argtypes = [vp, i64, vp, C.c_int, C.c_int, vp]
        L.oracle_ent_decode.restype = C.c_int
        _lib = L
    return _lib


def _p(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data


def tables():
    """Return the frozen tables (LOG2F, EXP2H, EXP2L, TGAM, K)."""
    log2f = np.zeros(4096, np.int32)
    eh = np.zeros(256, np.float32)
    el = np.zeros(256, np.float32)
    tg = np.zeros(256, np.float32)
    k = np.zeros((8, 8), np.int32)
    lib().oracle_tables(_p(log2f), _p(eh), _p(el), _p(tg), _p(k))
    return log2f, eh, el, tg, k


def keystat(rgbe: np.ndarray):
    rgbe = np.ascontiguousarray(rgbe, np.uint8)
    L = np.zeros(1, np.int64)
    N = np.zeros(1, np.int64)
    lib().oracle_keystat(_p(rgbe), rgbe.size // 4, _p(L), _p(N))
    return int(L[0]), int(N[0])


def key_params(lam: int, n: int):
    k = np.zeros(1, np.int32)
    f = np.zeros(1, np.int32)
    s = np.zeros(1, np.float32)
    lib().oracle_key_params(lam, n, _p(k), _p(f), _p(s))
    return int(k[0]), int(f[0]), np.float32(s[0])


def tmo(rgbe: np.ndarray, k_img: int, sigma, n_lit: int) -> np.ndarray:
    rgbe = np.ascontiguousarray(rgbe, np.uint8)
    H, W = rgbe.shape[:2]
    out = np.zeros((H, W, 3), np.uint8)
    lib().oracle_tmo(_p(rgbe), H, W, k_img, float(sigma), n_lit, _p(out))
    return out


def quant_table(q: int, chroma: bool) -> np.ndarray:
    out = np.zeros(64, np.int32)
    lib().oracle_quant_table(q, int(chroma), _p(out))
    return out.reshape(8, 8)


def fdct_block(block: np.ndarray) -> np.ndarray:
    a = np.ascontiguousarray(block, np.int32).reshape(64)
    o = np.zeros(64, np.int32)
    lib().oracle_fdct_block(_p(a), _p(o))
    return o.reshape(8, 8)


def idct_block(coef: np.ndarray) -> np.ndarray:
    a = np.ascontiguousarray(coef, np.int32).reshape(64)
    o = np.zeros(64, np.int32)
    lib().oracle_idct_block(_p(a), _p(o))
    return o.reshape(8, 8)


def quantise(F: int, Qt: int) -> int:
    return int(lib().oracle_quantise(F, Qt))


def base_layer(sdr0: np.ndarray, q: int, want_dct: bool = False):
    sdr0 = np.ascontiguousarray(sdr0, np.uint8)
    H, W = sdr0.shape[:2]
    S = np.zeros((H, W, 3), np.uint8)
    dct = None
    if want_dct:
        dct = np.zeros((3, (H + 7) // 8 * 8, (W + 7) // 8 * 8), np.int16)
    lib().oracle_base_layer(_p(sdr0), H, W, q, _p(S), _p(dct) if dct is not None else None)
    return (S, dct) if want_dct else S


def base_decode(dctq: np.ndarray, H: int, W: int, q: int) -> np.ndarray:
    """S from the quantised coefficients int16 [3][H8][W8] at quality q."""
    dctq = np.ascontiguousarray(dctq, np.int16)
    H8, W8 = (H + 7) // 8 * 8, (W + 7) // 8 * 8
    assert dctq.size == 3 * H8 * W8
    S = np.zeros((H, W, 3), np.uint8)
    if lib().oracle_base_decode(_p(dctq), H, W, q, _p(S)):
        raise ValueError("oracle_base_decode: bad arguments")
    return S


def gf(S: np.ndarray) -> np.ndarray:
    S = np.ascontiguousarray(S, np.uint8)
    H, W = S.shape[:2]
    out = np.zeros_like(S)
    lib().oracle_gf(_p(S), H, W, _p(out))
    return out


def sums(Sstar: np.ndarray, rgbe: np.ndarray) -> np.ndarray:
    Sstar = np.ascontiguousarray(Sstar, np.uint8)
    rgbe = np.ascontiguousarray(rgbe, np.uint8)
    out = np.zeros((256, 13), np.int64)
    lib().oracle_sums(_p(Sstar), _p(rgbe), rgbe.size // 4, _p(out))
    return out


def solve(sums_arr: np.ndarray):
    s = np.ascontiguousarray(sums_arr, np.int64)
    a = np.zeros((3, 256), np.int32)
    b = np.zeros((3, 256), np.int32)
    pr = np.zeros(256, np.uint8)
    lib().oracle_solve(_p(s), _p(a), _p(b), _p(pr))
    return a, b, pr


def mstar(a_q: int, b_q: int, s: int) -> int:
    return int(lib().oracle_mstar(a_q, b_q, s))


def resid(Sstar: np.ndarray, rgbe: np.ndarray, a_q: np.ndarray, b_q: np.ndarray) -> np.ndarray:
    Sstar = np.ascontiguousarray(Sstar, np.uint8)
    rgbe = np.ascontiguousarray(rgbe, np.uint8)
    npx = rgbe.size // 4
    out = np.zeros(7 * npx, np.uint8)
    lib().oracle_resid(_p(Sstar), _p(rgbe), npx, _p(np.ascontiguousarray(a_q, np.int32)),
                       _p(np.ascontiguousarray(b_q, np.int32)), _p(out))
    return out


def split_resid(buf: np.ndarray, H: int, W: int):
    """View a residual buffer as (int16 r[3][H][W], uint8 E[H][W])."""
    npx = H * W
    buf = np.asarray(buf).view(np.uint8).reshape(-1)
    r = buf[: 6 * npx].view(np.int16).reshape(3, H, W)
    E = buf[6 * npx: 7 * npx].reshape(H, W)
    return r, E


def encode_enh(rgbe: np.ndarray, q: int) -> dict:
    """Full encoder.  Returns a dict with sdr, a_q, b_q, present, sums,
    lambda_sum, n_lit, k_img, f_key, sigma, resid (7*H*W bytes)."""
    rgbe = np.ascontiguousarray(rgbe, np.uint8)
    H, W = rgbe.shape[:2]
    sdr = np.zeros((H, W, 3), np.uint8)
    a = np.zeros((3, 256), np.int32)
    b = np.zeros((3, 256), np.int32)
    pr = np.zeros(256, np.uint8)
    sm = np.zeros((256, 13), np.int64)
    par = np.zeros(5, np.int64)
    res = np.zeros(7 * H * W, np.uint8)
    rc = lib().oracle_encode_enh(_p(rgbe), H, W, q, _p(sdr), _p(a), _p(b), _p(pr), _p(sm), _p(par), _p(res))
    if rc != 0:
        raise ValueError("oracle_encode_enh failed with %d" % rc)
    return dict(sdr=sdr, a_q=a, b_q=b, present=pr, sums=sm, lambda_sum=int(par[0]), n_lit=int(par[1]),
                k_img=int(par[2]), f_key=int(par[3]),
                sigma=np.array([par[4]], np.uint32).view(np.float32)[0], resid=res)


def decode_enh(sdr: np.ndarray, a_q: np.ndarray, b_q: np.ndarray, resid: np.ndarray, H: int, W: int):
    sdr = np.ascontiguousarray(sdr, np.uint8)
    out = np.zeros((H, W, 4), np.uint8)
    rc = lib().oracle_decode_enh(_p(sdr), _p(np.ascontiguousarray(a_q, np.int32)),
                                 _p(np.ascontiguousarray(b_q, np.int32)),
                                 _p(np.ascontiguousarray(resid).view(np.uint8)), H, W, _p(out))
    if rc != 0:
        raise ValueError("oracle_decode_enh failed with %d" % rc)
    return out


def resid_hist(resid: np.ndarray, npx: int) -> np.ndarray:
    out = np.zeros((3, 511), np.int64)
    lib().oracle_resid_hist(_p(np.ascontiguousarray(resid).view(np.uint8)), npx, _p(out))
    return out


def bits_per_pixel(hist: np.ndarray) -> float:
    """Sum over channels of the zeroth-order entropy of the residual planes."""
    tot = 0.0
    for h in np.asarray(hist, np.float64):
        n = h.sum()
        if n <= 0:
            continue
        p = h[h > 0] / n
        tot += float(-(p * np.log2(p)).sum())
    return tot


# ---------------------------------------------------------------- learned estimator
def _blob(blob: bytes):
    return np.frombuffer(blob, np.uint8).copy()


def mlp_estimate(S: np.ndarray, rgbe: np.ndarray, k_img: int, blob: bytes) -> np.ndarray:
    S = np.ascontiguousarray(S, np.uint8)
    rgbe = np.ascontiguousarray(rgbe, np.uint8)
    H, W = S.shape[:2]
    out = np.zeros((H, W, 3), np.uint8)
    b = _blob(blob)
    rc = lib().oracle_mlp_estimate(_p(S), _p(rgbe), None, H, W, k_img, _p(b), _p(out))
    if rc:
        raise ValueError("bad model blob")
    return out


def log2q16(x: int) -> int:
    return int(lib().oracle_log2q16(int(x)))


def cross_cost(h, g) -> int:
    """Q16 code length of histogram h under the distribution of counts g
    (-1 when h has a value g never takes)."""
    h = np.ascontiguousarray(h, np.int64)
    g = np.ascontiguousarray(g, np.int64)
    return int(lib().oracle_cross_cost(_p(h), _p(g), int(g.sum()), h.size))


def hist_cost(h) -> int:
    h = np.ascontiguousarray(h, np.int64)
    return int(lib().oracle_hist_cost(_p(h), h.size))


def encode_learned(rgbe: np.ndarray, q: int, blob: bytes) -> dict:
    rgbe = np.ascontiguousarray(rgbe, np.uint8)
    H, W = rgbe.shape[:2]
    sdr = np.zeros((H, W, 3), np.uint8)
    a = np.zeros((3, 256), np.int32)
    b = np.zeros((3, 256), np.int32)
    pr = np.zeros(256, np.uint8)
    fl = np.zeros((3, 256), np.uint8)
    par = np.zeros(5, np.int64)
    res = np.zeros(7 * H * W, np.uint8)
    bb = _blob(blob)
    rc = lib().oracle_encode_learned(_p(rgbe), H, W, q, _p(bb), _p(sdr), _p(a), _p(b), _p(pr), _p(fl), _p(par),
                                     _p(res))
    if rc:
        raise ValueError("oracle_encode_learned failed with %d" % rc)
    return dict(sdr=sdr, a_q=a, b_q=b, present=pr, flag=fl, k_img=int(par[2]), resid=res)


def decode_learned(sdr, a_q, b_q, flag, k_img, blob, resid, H, W) -> np.ndarray:
    out = np.zeros((H, W, 4), np.uint8)
    bb = _blob(blob)
    rc = lib().oracle_decode_learned(_p(np.ascontiguousarray(sdr, np.uint8)), _p(np.ascontiguousarray(a_q, np.int32)),
                                     _p(np.ascontiguousarray(b_q, np.int32)), _p(np.ascontiguousarray(flag, np.uint8)),
                                     k_img, _p(bb), _p(np.ascontiguousarray(resid).view(np.uint8)), H, W, _p(out))
    if rc:
        raise ValueError("oracle_decode_learned failed with %d" % rc)
    return out


# ---------------------------------------------------------------- entropy code of the layer
ENT_HDR = 4136
ENT_HDR_CTX = 25640  # with the residual contexts (8 tables per channel)


def ent_freqs(h) -> np.ndarray:
    """Quantised frequencies (sum 2^15) of one table's symbol counts."""
    h = np.ascontiguousarray(h, np.int64)
    f = np.zeros(len(h), np.uint16)
    if lib().oracle_ent_freqs(_p(h), len(h), _p(f)):
        raise ValueError("oracle_ent_freqs: bad counts")
    return f


def ent_bound(H: int, W: int, log2_k: int = 8, contexts: bool = False) -> int:
    return int(lib().oracle_ent_bound(H, W, log2_k, 2 if contexts else 0))


def _sdr_arg(sdr, H, W):
    if sdr is None:
        return None, None
    s = np.ascontiguousarray(sdr, np.uint8).reshape(-1)
    assert s.size == 3 * H * W
    return s, _p(s)


def ent_encode(resid: np.ndarray, H: int, W: int, log2_k: int = 8, predict: bool = True, sdr=None) -> bytes:
    """Code stream of an enhancement layer (7 H W bytes); predict codes the
    exponent plane as differences from the left neighbour; with sdr (the
    decoded base layer, H x W x 3) each residual is coded with the table of
    its context sdr >> 5."""
    buf = np.ascontiguousarray(resid).view(np.uint8).reshape(-1)
    assert buf.size == 7 * H * W
    keep, sp = _sdr_arg(sdr, H, W)
    flags = (1 if predict else 0) | (2 if sdr is not None else 0)
    out = np.zeros(max(ent_bound(H, W, log2_k, sdr is not None), 1), np.uint8)
    n = lib().oracle_ent_encode(_p(buf), sp, H, W, log2_k, flags, _p(out), out.size)
    if n < 0:
        raise ValueError("oracle_ent_encode failed with %d" % n)
    return out[:n].tobytes()


def ent_decode(stream: bytes, H: int, W: int, sdr=None) -> np.ndarray:
    """Enhancement layer (7 H W bytes) from a code stream (sdr: the decoded
    base layer, needed for a stream with residual contexts)."""
    st = np.frombuffer(stream, np.uint8).copy()
    out = np.zeros(7 * H * W, np.uint8)
    keep, sp = _sdr_arg(sdr, H, W)
    rc = lib().oracle_ent_decode(_p(st), st.size, sp, H, W, _p(out))
    if rc:
        raise ValueError("oracle_ent_decode failed with %d" % rc)
    return out


# ---------------------------------------------------------------- ablations
def encode_mode(rgbe: np.ndarray, q: int, est: int, gf: bool) -> dict:
    """Encoder with estimator est (0 SLR per region, 2 one line per channel,
    3 M* = S) and the Gaussian filter on or off."""
    rgbe = np.ascontiguousarray(rgbe, np.uint8)
    H, W = rgbe.shape[:2]
    sdr = np.zeros((H, W, 3), np.uint8)
    a_q = np.zeros((3, 256), np.int32)
    b_q = np.zeros((3, 256), np.int32)
    present = np.zeros(256, np.uint8)
    resid = np.zeros(7 * H * W, np.uint8)
    rc = lib().oracle_encode_mode(_p(rgbe), H, W, q, est, int(bool(gf)), _p(sdr), _p(a_q), _p(b_q), _p(present),
                                  _p(resid))
    if rc:
        raise ValueError("oracle_encode_mode failed with %d" % rc)
    return {"sdr": sdr, "a_q": a_q, "b_q": b_q, "present": present, "resid": resid}


def decode_mode(sdr, a_q, b_q, resid, H: int, W: int, gf: bool) -> np.ndarray:
    out = np.zeros((H, W, 4), np.uint8)
    rc = lib().oracle_decode_mode(_p(np.ascontiguousarray(sdr, np.uint8)), _p(np.ascontiguousarray(a_q, np.int32)),
                                  _p(np.ascontiguousarray(b_q, np.int32)), _p(np.ascontiguousarray(resid)), H, W,
                                  int(bool(gf)), _p(out))
    if rc:
        raise ValueError("oracle_decode_mode failed with %d" % rc)
    return out


# ---------------------------------------------------------------- base-layer JPEG file
def jpeg_huff_table(freq):
    """Annex K.2 table of symbol counts freq[256]: (bits[1..16], huffval)."""
    f = np.ascontiguousarray(freq, np.int64)
    assert f.size == 256
    bits = np.zeros(17, np.uint8)
    hv = np.zeros(256, np.uint8)
    n = lib().oracle_jpeg_huff_table(_p(f), _p(bits), _p(hv))
    return bits[1:].copy(), hv[:n].copy()


def jpeg_write(dctq: np.ndarray, H: int, W: int, q: int) -> bytes:
    """Baseline JFIF file of the quantised coefficients int16 [3][H8][W8]."""
    dctq = np.ascontiguousarray(dctq, np.int16)
    cap = 4096 + 3 * dctq.size * 8
    out = np.zeros(cap, np.uint8)
    n = lib().oracle_jpeg_write(_p(dctq), H, W, q, _p(out), cap)
    if n < 0:
        raise ValueError("oracle_jpeg_write failed with %d" % n)
    return out[:n].tobytes()


"""Byte layout of the learned estimator's model blob (format only).

Little endian, 7512 bytes:
  u32 magic 'RDLM', u32 version 2, u64 hash (FNV-1a 64 of bytes 24..end),
  u32 reserved[2];
  i8  W1[32][32] (out, in)     i32 B1[32][32] (exponent bin, out)
  i32 m1[32], r1[32]
  i8  W2[32][32]               i32 B2[32], m2[32], r2[32]
  i8  W3[16][32]               i32 B3[16], m3[16], r3[16]
Version 2 semantics: hidden activations a = clamp((h m + 2^(r-1)) >> r, 0, 255)
(unsigned bytes; version 1 clamped at 127).  Value limits (checked by the
library when a model is loaded): multipliers in [1, 2^10), shifts in [1, 28],
|B1|, |B2|, |B3| <= 2^18, so every requantisation product stays below 2^31.
"""
from __future__ import annotations

import numpy as np

MAGIC = 0x4D4C4452
VERSION = 2
A_MAX = 255      # largest hidden activation
M_LIMIT = 1 << 10  # multipliers are below this
BYTES = 7512
FIELDS = [("W1", np.int8, (32, 32)), ("B1", np.int32, (32, 32)), ("m1", np.int32, (32,)), ("r1", np.int32, (32,)),
          ("W2", np.int8, (32, 32)), ("B2", np.int32, (32,)), ("m2", np.int32, (32,)), ("r2", np.int32, (32,)),
          ("W3", np.int8, (16, 32)), ("B3", np.int32, (16,)), ("m3", np.int32, (16,)), ("r3", np.int32, (16,))]


def fnv1a64(data: bytes) -> int:
    h = 0xCBF29CE484222325
    for b in data:
        h ^= b
        h = (h * 0x100000001B3) & 0xFFFFFFFFFFFFFFFF
    return h


def pack(params: dict) -> bytes:
    body = b"".join(np.ascontiguousarray(params[name], dtype).reshape(shape).astype("<" + np.dtype(dtype).str[1:])
                    .tobytes() for name, dtype, shape in FIELDS)
    head = np.array([MAGIC, VERSION], "<u4").tobytes() + np.array([fnv1a64(body)], "<u8").tobytes() + bytes(8)
    blob = head + body
    assert len(blob) == BYTES
    return blob


def unpack(blob: bytes) -> dict:
    out = {}
    off = 24
    for name, dtype, shape in FIELDS:
        n = int(np.prod(shape)) * np.dtype(dtype).itemsize
        out[name] = np.frombuffer(blob[off:off + n], dtype).reshape(shape).copy()
        off += n
    return out


def blob_hash(blob: bytes) -> int:
    return int(np.frombuffer(blob[8:16], "<u8")[0])

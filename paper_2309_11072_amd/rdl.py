"""Python binding of ``librdl.so`` (the C ABI in ``include/rdl.h``).

Argument marshalling only: every step of the encoder and decoder runs in the
HIP kernels behind the C ABI.  PyTorch provides device memory and streams.
If the library has not been built, or no GPU is present, calls fail loudly;
there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import json
import os

import numpy as np
import torch  # noqa: F401  (loads the HIP runtime before librdl.so binds to it)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librdl.so")

RDL_MAGIC = 0x314C4452
RDL_OK, RDL_EINVAL, RDL_EHIP, RDL_ECORRUPT, RDL_ENOMEM, RDL_EUNSUPPORTED = 0, -1, -2, -3, -4, -5

#: Byte layout of ``rdl_header`` (7232 bytes, little endian).
HEADER_DTYPE = np.dtype([
    ("magic", "<u4"), ("version", "<u4"), ("H", "<i4"), ("W", "<i4"), ("q", "<i4"),
    ("k_img", "<i4"), ("f_key", "<i4"), ("sigma", "<f4"), ("lambda_sum", "<i8"), ("n_lit", "<i8"),
    ("estimator", "<i4"), ("n_regions", "<i4"), ("model_hash", "<u8"),
    ("a_q", "<i4", (3, 256)), ("b_q", "<i4", (3, 256)), ("present", "u1", (256,)), ("flag", "u1", (3, 256)),
])
HEADER_BYTES = HEADER_DTYPE.itemsize

LAUNCH_DIRECT, LAUNCH_GRAPH = 0, 1

#: Images per call of the allocation-free encoder (its static scratch).
NOALLOC_MAX_IMAGES = 16

#: Encoder estimators (header field `estimator`, bits 0-3) and the filter-off bit.
EST_SLR, EST_LEARNED, EST_GLOBAL, EST_NONE = 0, 1, 2, 3
EST_GF_OFF = 16

#: Entropy code of the enhancement layer: fixed header bytes, default group size.
ENT_HEADER_BYTES = 4136
ENT_CTX_HEADER_BYTES = 25640  # with residual contexts (25 frequency tables)
ENT_LOG2K_DEFAULT = 8

# Exported symbols of include/rdl.h with their argument types.
_vp, _i, _i64p = C.c_void_p, C.c_int, C.c_void_p
_SIGS = {
    "rdl_create": ([C.POINTER(C.c_void_p), _i], _i),
    "rdl_destroy": ([_vp], None),
    "rdl_strerror": ([_i], C.c_char_p),
    "rdl_resid_bytes": ([_i, _i], C.c_size_t),
    "rdl_header_bytes": ([], C.c_size_t),
    "rdl_header_validate": ([_vp, _i, _i], _i),
    "rdl_encode_enh": ([_vp, _vp, _i, _i, _i, _vp, _vp, _vp, _vp], _i),
    "rdl_decode_enh": ([_vp, _vp, _vp, _vp, _i, _i, _vp, _vp, _vp], _i),
    "rdl_encode_batch": ([_vp, _vp, _i, _vp], _i),
    "rdl_encode_batch_noalloc": ([_vp, _vp, _i, _vp], _i),
    "rdl_decode_batch": ([_vp, _vp, _i, _vp], _i),
    "rdl_base_decode": ([_vp, _vp, _vp, _i, _i, _vp, _vp, _vp], _i),
    "rdl_resid_hist": ([_vp, _vp, _i, _i, _vp, _vp], _i),
    "rdl_jpeg_bound": ([_i, _i], C.c_size_t),
    "rdl_jpeg_encode": ([_vp, _vp, _i, _i, _i, _vp, C.c_size_t, _vp, _vp], _i),
    "rdl_ent_bound": ([_i, _i, _i], C.c_size_t),
    "rdl_ent_encode": ([_vp, _vp, _i, _i, _i, _vp, C.c_size_t, _vp, _vp], _i),
    "rdl_ent_decode": ([_vp, _vp, C.c_size_t, _vp, _i, _i, _vp, _vp, _vp], _i),
    "rdl_ent_bound_ctx": ([_i, _i, _i], C.c_size_t),
    "rdl_ent_encode_ctx": ([_vp, _vp, _vp, _i, _i, _i, _vp, C.c_size_t, _vp, _vp], _i),
    "rdl_ent_decode_ctx": ([_vp, _vp, C.c_size_t, _vp, _vp, _i, _i, _vp, _vp, _vp], _i),
    "rdl_stage_keystat": ([_vp, _vp, _i, _i, _vp, _vp], _i),
    "rdl_stage_tmo_base": ([_vp, _vp, _i, _i, _i, _vp, _vp, _vp, _vp, _vp], _i),
    "rdl_stage_fit": ([_vp, _vp, _vp, _i, _i, _i, _vp, _vp, _vp, _vp], _i),
    "rdl_stage_resid": ([_vp, _vp, _vp, _vp, _i, _i, _vp, _vp], _i),
    "rdl_profile_encode": ([_vp, _vp, _i, _i, _i, _vp, _vp, _vp, _i, _vp, _vp], _i),
    "rdl_autotune": ([_vp, _vp, _i, _i, _i, _vp, _vp, _vp, _i, _vp, _vp], _i),
    "rdl_get_tuning": ([_vp, _i, _i, _vp], _i),
    "rdl_check_recip": ([_vp, C.c_uint32, C.c_uint32, _vp, _vp], _i),
    "rdl_set_tuning": ([_vp, _i, _i, _i], _i),
    "rdl_set_launch_mode": ([_vp, _i], _i),
    "rdl_set_stage_timing": ([_vp, _i], _i),
    "rdl_stage_times": ([_vp, _vp, _vp], _i),
    "rdl_set_model": ([_vp, _vp, C.c_size_t], _i),
    "rdl_set_estimator": ([_vp, _i], _i),
    "rdl_set_gf": ([_vp, _i], _i),
    "rdl_set_ent_predict": ([_vp, _i], _i),
    "rdl_train_sample_bytes": ([], _i),
    "rdl_train_nparam": ([], _i),
    "rdl_train_samples": ([_vp, _vp, _vp, _i, _i, _i, _vp, C.c_int64, _vp, _vp], _i),
    "rdl_train_step": ([_vp, _vp, _vp, _vp, _vp, C.c_int64, C.c_int64, _i, C.c_float, _i, _vp, _vp], _i),
}

TUNE = ("fit_rows", "resid_rows", "fit_bins", "fit_waves")
STAGES = ("keystat", "tmo_base", "fit_sums", "solve", "resid")
KERNELS = ("k_keystat", "k_tmo_base", "k_fit_sums", "k_solve", "k_resid")
#: All encoder stages (rdl_stage_times order) and their kernels.  With the
#: learned estimator the "resid" stage runs k_resid_patch (k_learn has
#: already written the SLR residuals).
STAGES_ALL = STAGES + ("learn", "lhist", "select")
KERNELS_ALL = KERNELS + ("k_learn", "k_lhist", "k_select")
TIMING_MAX_CALLS = 64


class RdlImage(C.Structure):
    _fields_ = [("rgbe", C.c_void_p), ("H", C.c_int32), ("W", C.c_int32), ("q", C.c_int32),
                ("sdr", C.c_void_p), ("hdr", C.c_void_p), ("resid", C.c_void_p), ("dct", C.c_void_p)]


class RdlDImage(C.Structure):
    _fields_ = [("dct", C.c_void_p), ("sdr", C.c_void_p), ("hdr", C.c_void_p), ("resid", C.c_void_p),
                ("H", C.c_int32), ("W", C.c_int32), ("out_rgbe", C.c_void_p), ("status", C.c_void_p)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load librdl.so and declare its functions.  Raises if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise RuntimeError("librdl.so is not built (run __graft_entry__.build()); there is no CPU fallback")
        L = C.CDLL(path)
        for name, (args, res) in _SIGS.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


class RdlError(RuntimeError):
    def __init__(self, code: int, where: str):
        msg = load_library().rdl_strerror(code).decode()
        super().__init__("%s failed: %s (%d)" % (where, msg, code))
        self.code = code


def _chk(rc: int, where: str):
    if rc != RDL_OK:
        raise RdlError(rc, where)


def _ptr(t: torch.Tensor | None):
    if t is None:
        return None
    assert t.is_cuda and t.is_contiguous(), "device tensors must be contiguous"
    return t.data_ptr()


def _stream(stream):
    s = torch.cuda.current_stream() if stream is None else stream
    return s.cuda_stream


def header_from_bytes(buf) -> np.void:
    """Parse a header copied to the host (a uint8 tensor/array of 7232 bytes)."""
    if isinstance(buf, torch.Tensor):
        buf = buf.detach().cpu().numpy()
    return np.frombuffer(np.ascontiguousarray(buf).tobytes(), HEADER_DTYPE)[0]


def split_resid(resid: torch.Tensor, H: int, W: int):
    """(int16 r[3][H][W], uint8 E[H][W]) views of a residual buffer."""
    npx = H * W
    r = resid[: 6 * npx].view(torch.int16).view(3, H, W)
    E = resid[6 * npx: 7 * npx].view(H, W)
    return r, E


class Codec:
    """One rdl_ctx on one device."""

    def __init__(self, device: int = 0):
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device: the encoder runs only on the GPU")
        L = load_library()
        self.device = device
        h = C.c_void_p()
        _chk(L.rdl_create(C.byref(h), device), "rdl_create")
        self._h = h
        self._L = L

    def close(self):
        if getattr(self, "_h", None):
            self._L.rdl_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -------------------------------------------------------------- learned estimator
    def set_model(self, blob: bytes | None):
        """Load a model blob (host bytes) or clear it (None)."""
        if blob is None:
            _chk(self._L.rdl_set_model(self._h, None, 0), "rdl_set_model")
            return
        buf = C.create_string_buffer(bytes(blob), len(blob))
        _chk(self._L.rdl_set_model(self._h, buf, len(blob)), "rdl_set_model")

    def set_estimator(self, mode: int):
        """0: plain SLR; 1: learned estimate where it beats SLR per region;
        2: one SLR line per channel (ablation); 3: M* = S (ablation)."""
        _chk(self._L.rdl_set_estimator(self._h, int(mode)), "rdl_set_estimator")

    def set_gf(self, on: bool):
        """Gaussian-filter restoration of S before the estimate (on by default)."""
        _chk(self._L.rdl_set_gf(self._h, int(bool(on))), "rdl_set_gf")

    def set_ent_predict(self, on: bool):
        """Entropy code: the exponent plane as left differences (on by default)."""
        _chk(self._L.rdl_set_ent_predict(self._h, int(bool(on))), "rdl_set_ent_predict")

    # -------------------------------------------------------------- training
    def train_samples(self, rgbe: torch.Tensor, sdr: torch.Tensor, k_img: int, idx: torch.Tensor,
                      out: torch.Tensor | None = None, stream=None):
        """Sample records (uint8 [n, 32]) for the pixel indices idx (int64)."""
        H, W = int(rgbe.shape[0]), int(rgbe.shape[1])
        n = int(idx.numel())
        nb = self._L.rdl_train_sample_bytes()
        out = out if out is not None else torch.empty((n, nb), dtype=torch.uint8, device=rgbe.device)
        _chk(self._L.rdl_train_samples(self._h, _ptr(rgbe), _ptr(sdr), H, W, int(k_img), _ptr(idx), n, _ptr(out),
                                       _stream(stream)), "rdl_train_samples")
        return out

    def train_step(self, params, adam_m, adam_v, samples, base: int, batch: int, lr: float, step: int,
                   loss_out=None, stream=None):
        _chk(self._L.rdl_train_step(self._h, _ptr(params), _ptr(adam_m), _ptr(adam_v), _ptr(samples), int(base),
                                    int(samples.shape[0]), int(batch), float(lr), int(step), _ptr(loss_out),
                                    _stream(stream)), "rdl_train_step")

    # -------------------------------------------------------------- buffers
    def alloc_outputs(self, H: int, W: int):
        dev = torch.device("cuda", self.device)
        sdr = torch.empty((H, W, 3), dtype=torch.uint8, device=dev)
        hdr = torch.empty(HEADER_BYTES, dtype=torch.uint8, device=dev)
        resid = torch.empty(7 * H * W, dtype=torch.uint8, device=dev)
        return sdr, hdr, resid

    # -------------------------------------------------------------- encoder
    def encode_enh(self, rgbe: torch.Tensor, q: int, out=None, stream=None):
        """rgbe: uint8 [H, W, 4] on the device.  Returns (sdr, header, resid)."""
        H, W = int(rgbe.shape[0]), int(rgbe.shape[1])
        sdr, hdr, resid = out if out is not None else self.alloc_outputs(H, W)
        _chk(self._L.rdl_encode_enh(self._h, _ptr(rgbe), H, W, int(q), _ptr(sdr), _ptr(hdr), _ptr(resid),
                                    _stream(stream)), "rdl_encode_enh")
        return sdr, hdr, resid

    def encode_batch(self, items, stream=None):
        """items: list of (rgbe, q, sdr, hdr, resid) or (rgbe, q, sdr, hdr, resid, dct)
        device tensors (dct: the base layer's quantised coefficients, also written)."""
        arr = (RdlImage * len(items))()
        for k, it in enumerate(items):
            rgbe, q, sdr, hdr, resid = it[:5]
            dct = it[5] if len(it) > 5 else None
            arr[k] = RdlImage(_ptr(rgbe), int(rgbe.shape[0]), int(rgbe.shape[1]), int(q), _ptr(sdr), _ptr(hdr),
                              _ptr(resid), _ptr(dct))
        _chk(self._L.rdl_encode_batch(self._h, arr, len(items), _stream(stream)), "rdl_encode_batch")

    def encode_batch_noalloc(self, items, stream=None):
        """As encode_batch, through the allocation-free entry point (at most
        NOALLOC_MAX_IMAGES images, SLR-family estimators only)."""
        arr = (RdlImage * len(items))()
        for k, it in enumerate(items):
            rgbe, q, sdr, hdr, resid = it[:5]
            dct = it[5] if len(it) > 5 else None
            arr[k] = RdlImage(_ptr(rgbe), int(rgbe.shape[0]), int(rgbe.shape[1]), int(q), _ptr(sdr), _ptr(hdr),
                              _ptr(resid), _ptr(dct))
        _chk(self._L.rdl_encode_batch_noalloc(self._h, arr, len(items), _stream(stream)),
             "rdl_encode_batch_noalloc")

    def decode_batch(self, items, stream=None):
        """items: list of (dct or None, sdr, hdr, resid, out_rgbe, status or None) device
        tensors; with dct, sdr is written from the coefficients first."""
        arr = (RdlDImage * len(items))()
        for k, (dct, sdr, hdr, resid, out, status) in enumerate(items):
            arr[k] = RdlDImage(_ptr(dct), _ptr(sdr), _ptr(hdr), _ptr(resid), int(out.shape[0]), int(out.shape[1]),
                               _ptr(out), _ptr(status))
        _chk(self._L.rdl_decode_batch(self._h, arr, len(items), _stream(stream)), "rdl_decode_batch")

    def base_decode(self, dct: torch.Tensor, hdr: torch.Tensor, H: int, W: int, out: torch.Tensor | None = None,
                    status: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        """Base layer S (H x W x 3) from its quantised coefficients and the header's quality."""
        out = out if out is not None else torch.empty((H, W, 3), dtype=torch.uint8, device=dct.device)
        _chk(self._L.rdl_base_decode(self._h, _ptr(dct), _ptr(hdr), H, W, _ptr(out), _ptr(status), _stream(stream)),
             "rdl_base_decode")
        return out

    def decode_enh(self, sdr: torch.Tensor, hdr: torch.Tensor, resid: torch.Tensor, H: int, W: int,
                   out: torch.Tensor | None = None, status: torch.Tensor | None = None, stream=None):
        out = out if out is not None else torch.empty((H, W, 4), dtype=torch.uint8, device=sdr.device)
        _chk(self._L.rdl_decode_enh(self._h, _ptr(sdr), _ptr(hdr), _ptr(resid), H, W, _ptr(out), _ptr(status),
                                    _stream(stream)), "rdl_decode_enh")
        return out

    def resid_hist(self, resid: torch.Tensor, H: int, W: int, stream=None):
        hist = torch.empty((3, 511), dtype=torch.int64, device=resid.device)
        _chk(self._L.rdl_resid_hist(self._h, _ptr(resid), H, W, _ptr(hist), _stream(stream)), "rdl_resid_hist")
        return hist

    # ------------------------------------------------- base layer as a JPEG file
    def jpeg_encode_into(self, dct: torch.Tensor, H: int, W: int, q: int, out: torch.Tensor, out_len: torch.Tensor,
                         stream=None) -> None:
        """JFIF file of the quantised coefficients into out (uint8, >= rdl_jpeg_bound
        bytes); its length to out_len (one int64 on the device).  Does not synchronise."""
        assert out.dtype == torch.uint8 and out_len.dtype == torch.int64 and out_len.numel() == 1
        _chk(self._L.rdl_jpeg_encode(self._h, _ptr(dct), H, W, int(q), _ptr(out), out.numel(), _ptr(out_len),
                                     _stream(stream)), "rdl_jpeg_encode")

    def encode_files(self, rgbe: torch.Tensor, q: int, log2_k: int = 8, stream=None):
        """The dual-layer files of one image: (JPEG file of the base layer, device
        header, entropy-coded enhancement layer); synchronises."""
        H, W = int(rgbe.shape[0]), int(rgbe.shape[1])
        sdr, hdr, resid = self.alloc_outputs(H, W)
        dct = torch.empty((3, (H + 7) // 8 * 8, (W + 7) // 8 * 8), dtype=torch.int16, device=rgbe.device)
        self.encode_batch([(rgbe, q, sdr, hdr, resid, dct)], stream)
        return self.jpeg_encode(dct, H, W, q, stream), hdr, self.ent_encode(resid, H, W, log2_k, stream)

    def jpeg_bound(self, H: int, W: int) -> int:
        return int(self._L.rdl_jpeg_bound(H, W))

    def jpeg_encode(self, dct: torch.Tensor, H: int, W: int, q: int, stream=None) -> torch.Tensor:
        """The JFIF file (uint8 device tensor, trimmed; synchronises)."""
        out = torch.empty(self.jpeg_bound(H, W), dtype=torch.uint8, device=dct.device)
        n = torch.zeros(1, dtype=torch.int64, device=dct.device)
        self.jpeg_encode_into(dct, H, W, q, out, n, stream)
        return out[:int(n.item())]

    # ------------------------------------------------- entropy code of the layer
    # sdr (the decoded base layer, uint8 H x W x 3 on the device) selects the
    # stream with residual contexts: each residual coded with the table of its
    # context sdr >> 5.
    def ent_bound(self, H: int, W: int, log2_k: int = ENT_LOG2K_DEFAULT, contexts: bool = False) -> int:
        fn = self._L.rdl_ent_bound_ctx if contexts else self._L.rdl_ent_bound
        return int(fn(H, W, log2_k))

    def ent_encode_into(self, resid: torch.Tensor, H: int, W: int, out: torch.Tensor, out_len: torch.Tensor,
                        log2_k: int = ENT_LOG2K_DEFAULT, stream=None, sdr: torch.Tensor | None = None) -> None:
        """Code stream of resid into out (uint8, >= ent_bound bytes); its length
        goes to out_len (one int64 on the device).  Does not synchronise."""
        assert out.dtype == torch.uint8 and out_len.dtype == torch.int64 and out_len.numel() == 1
        if sdr is None:
            _chk(self._L.rdl_ent_encode(self._h, _ptr(resid), H, W, int(log2_k), _ptr(out), out.numel(),
                                        _ptr(out_len), _stream(stream)), "rdl_ent_encode")
        else:
            assert sdr.dtype == torch.uint8 and sdr.numel() == 3 * H * W and sdr.is_contiguous()
            _chk(self._L.rdl_ent_encode_ctx(self._h, _ptr(resid), _ptr(sdr), H, W, int(log2_k), _ptr(out),
                                            out.numel(), _ptr(out_len), _stream(stream)), "rdl_ent_encode_ctx")

    def ent_encode(self, resid: torch.Tensor, H: int, W: int, log2_k: int = ENT_LOG2K_DEFAULT,
                   stream=None, sdr: torch.Tensor | None = None) -> torch.Tensor:
        """Code stream of an enhancement layer, trimmed to its length (synchronises)."""
        out = torch.empty(self.ent_bound(H, W, log2_k, sdr is not None), dtype=torch.uint8, device=resid.device)
        n = torch.zeros(1, dtype=torch.int64, device=resid.device)
        self.ent_encode_into(resid, H, W, out, n, log2_k, stream, sdr)
        length = int(n.item())
        if length == 0:
            raise RdlError(RDL_EINVAL, "rdl_ent_encode (residual outside [-255, 255])")
        return out[:length]

    def ent_decode(self, code: torch.Tensor, H: int, W: int, out: torch.Tensor | None = None,
                   status: torch.Tensor | None = None, header: np.ndarray | None = None, stream=None,
                   sdr: torch.Tensor | None = None) -> torch.Tensor:
        """Enhancement layer (7 H W bytes) from a device code stream.  header: a
        host copy of the stream's first ENT_HEADER_BYTES bytes (ENT_CTX_HEADER_BYTES
        with sdr; read from the device, synchronously, when not given)."""
        nh = ENT_HEADER_BYTES if sdr is None else ENT_CTX_HEADER_BYTES
        hdr = np.ascontiguousarray(header if header is not None else code[:nh].cpu().numpy())
        assert hdr.dtype == np.uint8 and hdr.size >= nh
        if out is None:
            out = torch.empty(7 * H * W, dtype=torch.uint8, device=code.device)
        if sdr is None:
            _chk(self._L.rdl_ent_decode(self._h, _ptr(code), code.numel(), hdr.ctypes.data, H, W, _ptr(out),
                                        _ptr(status), _stream(stream)), "rdl_ent_decode")
        else:
            assert sdr.dtype == torch.uint8 and sdr.numel() == 3 * H * W and sdr.is_contiguous()
            _chk(self._L.rdl_ent_decode_ctx(self._h, _ptr(code), code.numel(), hdr.ctypes.data, _ptr(sdr), H, W,
                                            _ptr(out), _ptr(status), _stream(stream)), "rdl_ent_decode_ctx")
        return out

    def profile_encode(self, rgbe: torch.Tensor, q: int, out, reps: int = 20, stream=None):
        """Mean duration in ms of each stage kernel (HIP events on the stream)."""
        H, W = int(rgbe.shape[0]), int(rgbe.shape[1])
        sdr, hdr, resid = out
        ms = (C.c_float * len(STAGES))()
        _chk(self._L.rdl_profile_encode(self._h, _ptr(rgbe), H, W, int(q), _ptr(sdr), _ptr(hdr), _ptr(resid), int(reps),
                                        ms, _stream(stream)), "rdl_profile_encode")
        return dict(zip(STAGES, [float(v) for v in ms]))

    # -------------------------------------------------------------- stages
    def autotune(self, rgbe: torch.Tensor, q: int, out, reps: int = 10, stream=None) -> dict:
        """Times the fit and the residual kernels on this image with each
        strip height, keeps the fastest for its size class, returns them."""
        H, W = int(rgbe.shape[0]), int(rgbe.shape[1])
        sdr, hdr, resid = out
        best = (C.c_int * len(TUNE))()
        _chk(self._L.rdl_autotune(self._h, _ptr(rgbe), H, W, int(q), _ptr(sdr), _ptr(hdr), _ptr(resid), int(reps),
                                  best, _stream(stream)), "rdl_autotune")
        return dict(zip(TUNE, [int(v) for v in best]))

    def check_recip(self, lo_bits: int, hi_bits: int, stream=None) -> int:
        """Number of floats with bits in [lo_bits, hi_bits) whose kernel
        reciprocal differs from IEEE division."""
        n = C.c_uint64(0)
        _chk(self._L.rdl_check_recip(self._h, lo_bits, hi_bits, C.byref(n), _stream(stream)), "rdl_check_recip")
        return int(n.value)

    def get_tuning(self) -> dict:
        """{parameter: [value of size class floor(log2(H W)) for 0..31]}."""
        out = {}
        v = C.c_int(0)
        for p, name in enumerate(TUNE):
            row = []
            for k in range(32):
                _chk(self._L.rdl_get_tuning(self._h, p, k, C.byref(v)), "rdl_get_tuning")
                row.append(int(v.value))
            out[name] = row
        return out

    def set_stage_timing(self, on: bool) -> None:
        """Record HIP events around every stage kernel of later direct encodes."""
        _chk(self._L.rdl_set_stage_timing(self._h, int(bool(on))), "rdl_set_stage_timing")

    def stage_times(self):
        """Mean stage durations (ms) over the recorded encodes, and their count;
        starts a new recording."""
        ms = (C.c_float * len(STAGES_ALL))()
        n = C.c_int(0)
        _chk(self._L.rdl_stage_times(self._h, ms, C.byref(n)), "rdl_stage_times")
        return {k: float(v) for k, v in zip(STAGES_ALL, ms)}, int(n.value)

    def set_launch_mode(self, graph: bool) -> None:
        """False (default): one launch per stage kernel; True: each encoder
        plan is captured in a HIP graph at first use and replayed."""
        _chk(self._L.rdl_set_launch_mode(self._h, LAUNCH_GRAPH if graph else LAUNCH_DIRECT), "rdl_set_launch_mode")

    def set_tuning(self, table: dict) -> None:
        for p, name in enumerate(TUNE):
            for k, v in enumerate(table.get(name, [])):
                _chk(self._L.rdl_set_tuning(self._h, p, k, int(v)), "rdl_set_tuning")

    def save_tuning(self, path: str) -> None:
        with open(path, "w") as fh:
            json.dump(self.get_tuning(), fh)

    def load_tuning(self, path: str) -> None:
        with open(path) as fh:
            self.set_tuning(json.load(fh))

    def stage_keystat(self, rgbe: torch.Tensor, stream=None):
        out = torch.empty(2, dtype=torch.int64, device=rgbe.device)
        _chk(self._L.rdl_stage_keystat(self._h, _ptr(rgbe), int(rgbe.shape[0]), int(rgbe.shape[1]), _ptr(out),
                                       _stream(stream)), "rdl_stage_keystat")
        return out

    def stage_tmo_base(self, rgbe: torch.Tensor, q: int, keystat: torch.Tensor, want_sdr0=False, want_dct=False,
                       stream=None):
        H, W = int(rgbe.shape[0]), int(rgbe.shape[1])
        dev = rgbe.device
        sdr = torch.empty((H, W, 3), dtype=torch.uint8, device=dev)
        sdr0 = torch.empty((H, W, 3), dtype=torch.uint8, device=dev) if want_sdr0 else None
        dct = None
        if want_dct:
            dct = torch.empty((3, (H + 7) // 8 * 8, (W + 7) // 8 * 8), dtype=torch.int16, device=dev)
        _chk(self._L.rdl_stage_tmo_base(self._h, _ptr(rgbe), H, W, int(q), _ptr(keystat), _ptr(sdr0), _ptr(sdr),
                                        _ptr(dct), _stream(stream)), "rdl_stage_tmo_base")
        return sdr, sdr0, dct

    def stage_fit(self, rgbe: torch.Tensor, sdr: torch.Tensor, q: int, keystat: torch.Tensor | None = None,
                  stream=None):
        H, W = int(rgbe.shape[0]), int(rgbe.shape[1])
        sums = torch.empty((256, 13), dtype=torch.int64, device=rgbe.device)
        hdr = torch.empty(HEADER_BYTES, dtype=torch.uint8, device=rgbe.device)
        _chk(self._L.rdl_stage_fit(self._h, _ptr(rgbe), _ptr(sdr), H, W, int(q), _ptr(keystat), _ptr(sums), _ptr(hdr),
                                   _stream(stream)), "rdl_stage_fit")
        return sums, hdr

    def stage_resid(self, rgbe: torch.Tensor, sdr: torch.Tensor, hdr: torch.Tensor, stream=None):
        H, W = int(rgbe.shape[0]), int(rgbe.shape[1])
        resid = torch.empty(7 * H * W, dtype=torch.uint8, device=rgbe.device)
        _chk(self._L.rdl_stage_resid(self._h, _ptr(rgbe), _ptr(sdr), _ptr(hdr), H, W, _ptr(resid), _stream(stream)),
             "rdl_stage_resid")
        return resid

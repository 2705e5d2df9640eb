"""Python binding of ``liblsim.so`` (include/lsim.h).

Argument marshalling only: every function checks tensor devices, dtypes and
shapes, passes raw device pointers and torch's current HIP stream to the
C-ABI, and raises ``LsimError`` on a non-OK status.  All computation happens
in the library's HIP kernels; torch provides device memory and streams.
There is no CPU fallback: without the built library every call raises.
"""
from __future__ import annotations

import ctypes
import os

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "liblsim.so")

SPA_F32, OMS_I8, NMS_F32 = 0, 1, 2
DEMAP_EXACT, DEMAP_MAXLOG = 0, 1
FAMILY_11N, FAMILY_BG = 0, 1
LAYERS_NATURAL, LAYERS_GROUPED, LAYERS_CUSTOM = 0, 1, 2
NDM_PARAMS = 4676

_lib = None


class LsimError(RuntimeError):
    pass


class CodeInfo(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int64), ("n_mother", ctypes.c_int64), ("e_tx", ctypes.c_int64),
                ("n_dec", ctypes.c_int64), ("m_dec", ctypes.c_int64), ("n_edges", ctypes.c_int64),
                ("Z", ctypes.c_int32), ("mb", ctypes.c_int32), ("nb", ctypes.c_int32),
                ("kb", ctypes.c_int32), ("rows", ctypes.c_int32), ("cols", ctypes.c_int32),
                ("n_punct_cols", ctypes.c_int32), ("max_row_deg", ctypes.c_int32),
                ("max_col_deg", ctypes.c_int32), ("n_shared_cols", ctypes.c_int32),
                ("n_private_rows", ctypes.c_int32)]


class DecodeParams(ctypes.Structure):
    _fields_ = [("algo", ctypes.c_int), ("iters", ctypes.c_int), ("offset", ctypes.c_float),
                ("alpha", ctypes.c_float), ("llr_max", ctypes.c_float), ("sat", ctypes.c_int),
                ("threads", ctypes.c_int), ("lds_rows", ctypes.c_int)]


_P = ctypes.c_void_p
_I = ctypes.c_int
_I64 = ctypes.c_int64
_U64 = ctypes.c_uint64
_F = ctypes.c_float
_SZ = ctypes.c_size_t

_SIGS = {
    "lsim_code_create": [_P, _I, _I, _I, _I, _I, _I64, ctypes.POINTER(_P)],
    "lsim_code_destroy": [_P],
    "lsim_code_query": [_P, ctypes.POINTER(CodeInfo)],
    "lsim_code_set_layer_order": [_P, _I, _P],
    "lsim_code_layer_order": [_P, _P, ctypes.POINTER(ctypes.c_int)],
    "lsim_source_bits": [_U64, _I64, _I64, _I64, _P, _P],
    "lsim_encode": [_P, _P, _I64, _P, _P],
    "lsim_map_awgn": [_P, _I, _P, _P, _U64, _I64, _I64, _P, _P],
    "lsim_map_points": [_P, _I, _P, _P, _P, _U64, _I64, _I64, _P, _P],
    "lsim_demap_prior": [_I, _I, _P, _P, _P, _I64, _I64, _I, _P, _P],
    "lsim_map_awgn_bits": [_I, _P, _I64, _I64, _P, _U64, _I64, _I64, _P, _P],
    "lsim_polar_construct": [_I, _I, ctypes.c_double, _P],
    "lsim_polar_create": [_I, _P, _I, ctypes.c_uint32, ctypes.POINTER(_P)],
    "lsim_polar_destroy": [_P],
    "lsim_polar_query": [_P, ctypes.POINTER(_I), ctypes.POINTER(_I), ctypes.POINTER(_I)],
    "lsim_polar_encode": [_P, _P, _I64, _P, _P],
    "lsim_polar_decode": [_P, _I, _I, _P, _I64, _P, _P, _P],
    "lsim_apriori_llrs": [_P, _P, _P, _U64, _I64, _I64, _P, _P],
    "lsim_mutual_info": [_P, _I64, _P, _I64, _I64, _I64, _P, _I, _P, _P, _P],
    "lsim_extrinsic": [_P, _P, _P, _F, _I64, _P, _P],
    "lsim_points_workspace": [_P, _I, _I64, ctypes.POINTER(_SZ)],
    "lsim_points_grad": [_P, _I, _P, _P, _P, _I64, _P, _P, _SZ, _P],
    "lsim_demap": [_I, _I, _P, _P, _I64, _I64, _P, _P],
    "lsim_demap_q8": [_I, _I, _P, _P, _I64, _I64, _F, _I, _P, _P],
    "lsim_quantize": [_P, _I64, _F, _I, _P, _P],
    "lsim_decode_workspace": [_P, ctypes.POINTER(DecodeParams), _I64, ctypes.POINTER(_SZ)],
    "lsim_decode": [_P, ctypes.POINTER(DecodeParams), _P, _I64, _P, _P, _P, _SZ, _P],
    "lsim_decode_launch": [_P, ctypes.POINTER(DecodeParams), ctypes.POINTER(_I), ctypes.POINTER(_I),
                           ctypes.POINTER(_I), ctypes.POINTER(_I)],
    "lsim_decode_noalloc": [_P, ctypes.POINTER(DecodeParams), _P, _I64, _P, _P, _P],
    "lsim_decode_state": [_P, ctypes.POINTER(DecodeParams), _P, _I64, _P, _P, _P, _P, _P, _SZ, _P],
    "lsim_count_errors": [_P, _I64, _P, _I64, _I64, _P, _I, _P, _P],
    "lsim_syndrome": [_P, _P, _I64, _I64, _P, _P],
    "lsim_hard_bits": [_P, _I64, _I64, _I64, _P, _P],
    "lsim_ebn0_to_n0": [_P, _I64, ctypes.c_double, _I, _P],
    "lsim_probe": [_I, _P, _P, _I64, _I, _I, ctypes.POINTER(_I64), _P],
    "lsim_mixed_plan_create": [_P, _P, _I, ctypes.POINTER(DecodeParams), _P, _I, ctypes.POINTER(_P)],
    "lsim_mixed_plan_destroy": [_P],
    "lsim_mixed_workspace": [_P, ctypes.POINTER(_SZ)],
    "lsim_mixed_decode": [_P, _P, _P, _P, _P, _SZ, _I, _P],
    "lsim_wbp_forward": [_P, _I, _P, _P, _I64, _F, _P, _P, _P],
    "lsim_wbp_workspace": [_P, _I, _I64, ctypes.POINTER(_SZ)],
    "lsim_wbp_backward": [_P, _I, _P, _P, _P, _I64, _F, _P, _P, _P, _P, _SZ, _P],
    "lsim_ndm_forward": [_P, _P, _P, _I64, _I64, _P, _P],
    "lsim_ndm_workspace": [_I64, _I64, ctypes.POINTER(_SZ)],
    "lsim_ndm_backward": [_P, _P, _P, _P, _I64, _I64, _P, _P, _P, _SZ, _P],
    "lsim_bce_workspace": [_I64, _I64, ctypes.POINTER(_SZ)],
    "lsim_bce_grad": [_P, _P, _I64, _I64, _I64, _F, _P, _P, _P, _SZ, _P],
    "lsim_adam_step": [_P, _P, _P, _P, _I64, _F, _F, _F, _F, _I, _P],
    "lsim_link_run": [_P, _P],
    "lsim_last_error": [],
    "lsim_version": [],
}


def lib():
    """Load the library once; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise LsimError(f"{LIB_PATH} is missing: run paper_2203_11854_amd.build.build() first")
    L = ctypes.CDLL(LIB_PATH)
    for name, args in _SIGS.items():
        fn = getattr(L, name, None)
        if fn is None:
            continue
        fn.argtypes = args
        fn.restype = None if name.endswith(("_destroy",)) else (
            ctypes.c_char_p if name in ("lsim_last_error", "lsim_version") else ctypes.c_int)
    _lib = L
    return L


def _call(name, *args):
    st = getattr(lib(), name)(*args)
    if st != 0:
        msg = lib().lsim_last_error().decode()
        raise LsimError(f"{name}: status {st}: {msg}")


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t, dtype=None, name="tensor"):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise LsimError(f"{name} must be a device tensor")
    if dtype is not None and t.dtype != dtype:
        raise LsimError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise LsimError(f"{name} must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _empty(shape, dtype, device):
    return torch.empty(shape, dtype=dtype, device=device)


# ------------------------------------------------------------------ codes

class Code:
    """A QC-LDPC code on the current device (lsim_code_create)."""

    def __init__(self, base, Z: int, family: str, n_punct_cols: int, e_tx: int):
        import numpy as np
        arr = np.ascontiguousarray(np.asarray(base, dtype=np.int16))
        mb, nb = arr.shape
        fam = FAMILY_11N if family == "11n" else FAMILY_BG
        h = ctypes.c_void_p()
        _call("lsim_code_create", arr.ctypes.data_as(ctypes.c_void_p), mb, nb, Z, fam,
              n_punct_cols, e_tx, ctypes.byref(h))
        self._h = h
        info = CodeInfo()
        _call("lsim_code_query", h, ctypes.byref(info))
        self.info = info
        for f, _ in CodeInfo._fields_:
            setattr(self, f, getattr(info, f))
        self.E = info.n_edges

    @classmethod
    def from_qcbase(cls, qb, e_tx: int) -> "Code":
        return cls(qb.base, qb.Z, qb.family, qb.n_punct_cols, e_tx)

    @property
    def handle(self):
        return self._h

    @property
    def tx_lo(self) -> int:
        """First transmitted mother-code bit (lsim_code_create's rate matching)."""
        return self.n_punct_cols * self.Z

    def set_layer_order(self, order="natural"):
        """Layered decoder's row order (lsim_code_set_layer_order): "natural",
        "grouped" or a permutation of range(rows).  Waits for the device
        first: the table must not change under a decode in flight."""
        import numpy as np
        torch.cuda.synchronize()
        if isinstance(order, str):
            mode = {"natural": LAYERS_NATURAL, "grouped": LAYERS_GROUPED}[order]
            _call("lsim_code_set_layer_order", self._h, mode, None)
        else:
            arr = np.ascontiguousarray(np.asarray(order, dtype=np.int32))
            if arr.shape != (self.rows,):
                raise LsimError(f"layer order needs {self.rows} rows")
            _call("lsim_code_set_layer_order", self._h, LAYERS_CUSTOM,
                  arr.ctypes.data_as(ctypes.c_void_p))

    def layer_order(self):
        """(order as a list of rows, workgroup barriers per iteration)."""
        import numpy as np
        arr = np.zeros(self.rows, dtype=np.int32)
        nb = ctypes.c_int()
        _call("lsim_code_layer_order", self._h, arr.ctypes.data_as(ctypes.c_void_p), ctypes.byref(nb))
        return arr.tolist(), nb.value

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.lsim_code_destroy(h)
            self._h = None


# --------------------------------------------------------------- pipeline

def source_bits(seed: int, cw0: int, B: int, k: int, device="cuda", out=None):
    u = out if out is not None else _empty((B, k), torch.uint8, device)
    _call("lsim_source_bits", seed, cw0, B, k, _ptr(u, torch.uint8, "u"), _stream())
    return u


def encode(code: Code, u, out=None):
    B = u.shape[0]
    c = out if out is not None else _empty((B, code.n_mother), torch.uint8, u.device)
    _call("lsim_encode", code.handle, _ptr(u, torch.uint8, "u"), B, _ptr(c, torch.uint8, "c"), _stream())
    return c


def map_awgn(code: Code, m: int, c, no, seed: int, cw0: int, out=None):
    B = c.shape[0]
    S = code.e_tx // m
    y = out if out is not None else _empty((B, S, 2), torch.float32, c.device)
    _call("lsim_map_awgn", code.handle, m, _ptr(c, torch.uint8, "c"), _ptr(no, torch.float32, "no"),
          seed, cw0, B, _ptr(y, torch.float32, "y"), _stream())
    return y


def map_points(code: Code, m: int, points, c, no, seed: int, cw0: int, out=None):
    """Trainable-constellation mapper + AWGN: points f32[2^m][2]."""
    B = c.shape[0]
    S = code.e_tx // m
    y = out if out is not None else _empty((B, S, 2), torch.float32, c.device)
    _call("lsim_map_points", code.handle, m, _ptr(points, torch.float32, "points"),
          _ptr(c, torch.uint8, "c"), _ptr(no, torch.float32, "no"), seed, cw0, B,
          _ptr(y, torch.float32, "y"), _stream())
    return y


def points_grad(code: Code, m: int, points, c, gy, out=None, work=None):
    """dLoss/dpoints f32[2^m][2] from dLoss/dy f32[B][S][2]."""
    B = c.shape[0]
    g = out if out is not None else _empty((1 << m, 2), torch.float32, gy.device)
    work, nbytes = _work(points_workspace(code, m, B), gy.device, work)
    _call("lsim_points_grad", code.handle, m, _ptr(points, torch.float32, "points"),
          _ptr(c, torch.uint8, "c"), _ptr(gy, torch.float32, "gy"), B,
          _ptr(g, torch.float32, "gpoints"), _ptr(work, None, "work"), nbytes, _stream())
    return g


def map_awgn_bits(m: int, bits, no, seed: int, cw0: int, n: int | None = None, out=None):
    """Mapper + AWGN on rows of bits (the first n columns of each row)."""
    B = bits.shape[0]
    n = bits.shape[1] if n is None else n
    if bits.dtype != torch.uint8 or bits.stride(1) != 1:
        raise LsimError("bits must be u8 with unit column stride")
    y = out if out is not None else _empty((B, n // m, 2), torch.float32, bits.device)
    _call("lsim_map_awgn_bits", m, ctypes.c_void_p(bits.data_ptr()), bits.stride(0), n,
          _ptr(no, torch.float32, "no"), seed, cw0, B, _ptr(y, torch.float32, "y"), _stream())
    return y


def polar_construct(n: int, K: int, design_ebn0_db: float):
    """Information mask (numpy u8[2^n]) by Bhattacharyya parameters."""
    import numpy as np
    mask = np.zeros(1 << n, dtype=np.uint8)
    _call("lsim_polar_construct", n, K, design_ebn0_db, mask.ctypes.data_as(ctypes.c_void_p))
    return mask


class PolarCode:
    """A Polar code on the current device (lsim_polar_create)."""

    def __init__(self, n: int, mask, crc_degree: int = 0, crc_poly: int = 0):
        import numpy as np
        m = np.ascontiguousarray(np.asarray(mask, dtype=np.uint8))
        if m.size != (1 << n):
            raise LsimError("mask must have 2^n entries")
        h = ctypes.c_void_p()
        _call("lsim_polar_create", n, m.ctypes.data_as(ctypes.c_void_p), crc_degree, crc_poly,
              ctypes.byref(h))
        self._h = h
        N, K, r = _I(), _I(), _I()
        _call("lsim_polar_query", h, ctypes.byref(N), ctypes.byref(K), ctypes.byref(r))
        self.n, self.N, self.K, self.r = n, N.value, K.value, r.value
        self.D = self.K - self.r

    @property
    def handle(self):
        return self._h

    def encode(self, data, out=None):
        B = data.shape[0]
        x = out if out is not None else _empty((B, self.N), torch.uint8, data.device)
        _call("lsim_polar_encode", self._h, _ptr(data, torch.uint8, "data"), B,
              _ptr(x, torch.uint8, "x"), _stream())
        return x

    def decode(self, llr, list_size: int = 1, use_crc: bool = False, bits=None, pm=None,
               want_pm: bool = False):
        B = llr.shape[0]
        if bits is None:
            bits = _empty((B, self.D), torch.uint8, llr.device)
        if want_pm and pm is None:
            pm = _empty((B, list_size), torch.float32, llr.device)
        _call("lsim_polar_decode", self._h, list_size, int(bool(use_crc)),
              _ptr(llr, torch.float32, "llr"), B, _ptr(bits, torch.uint8, "bits"),
              _ptr(pm, torch.float32, "pm") if pm is not None else None, _stream())
        return (bits, pm) if want_pm else bits

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.lsim_polar_destroy(h)
            self._h = None


def demap(m: int, method: int, y, no, out=None):
    B, S = y.shape[0], y.shape[1]
    L = out if out is not None else _empty((B, S * m), torch.float32, y.device)
    _call("lsim_demap", m, method, _ptr(y, torch.float32, "y"), _ptr(no, torch.float32, "no"), B, S,
          _ptr(L, torch.float32, "llr"), _stream())
    return L


def demap_prior(m: int, method: int, y, no, la, extrinsic: bool = True, out=None):
    """Demapper with prior: extrinsic (default) or a-posteriori LLRs."""
    B, S = y.shape[0], y.shape[1]
    L = out if out is not None else _empty((B, S * m), torch.float32, y.device)
    _call("lsim_demap_prior", m, method, _ptr(y, torch.float32, "y"), _ptr(no, torch.float32, "no"),
          _ptr(la, torch.float32, "la"), B, S, int(bool(extrinsic)), _ptr(L, torch.float32, "llr"),
          _stream())
    return L


def apriori_llrs(code: Code, c, sigma, seed: int, cw0: int, out=None):
    """Consistent Gaussian a-priori LLRs f32[B][e_tx] of the transmitted bits."""
    B = c.shape[0]
    la = out if out is not None else _empty((B, code.e_tx), torch.float32, c.device)
    _call("lsim_apriori_llrs", code.handle, _ptr(c, torch.uint8, "c"),
          _ptr(sigma, torch.float32, "sigma"), seed, cw0, B, _ptr(la, torch.float32, "la"),
          _stream())
    return la


def mutual_info(llr, c, bins=None, nbins: int = 1, mi_cw=None, mi_bins=None, want_bins=True):
    """(per-row MI f32[B], per-bin mean MI f64[nbins] or None); rows of c
    may be wider than llr's (only the first n columns are read)."""
    B, n = llr.shape
    if c.dtype != torch.uint8 or c.stride(1) != 1 or llr.stride(1) != 1:
        raise LsimError("llr f32 and labels u8 need unit column stride")
    if mi_cw is None:
        mi_cw = _empty((B,), torch.float32, llr.device)
    if want_bins and mi_bins is None:
        mi_bins = _empty((nbins,), torch.float64, llr.device)
    _call("lsim_mutual_info", _ptr(llr, torch.float32, "llr"), llr.stride(0),
          ctypes.c_void_p(c.data_ptr()), c.stride(0), B, n,
          _ptr(bins, torch.int32, "bins") if bins is not None else None, nbins,
          _ptr(mi_cw, torch.float32, "mi_cw"),
          _ptr(mi_bins, torch.float64, "mi_bins") if want_bins else None, _stream())
    return mi_cw, (mi_bins if want_bins else None)


def extrinsic(code: Code, app, llr_in, llr_max: float = 20.0, out=None):
    """Decoder extrinsic on the transmitted bits: L_post[tx] - L_in, L_in
    clamped to +-llr_max as the float decoders clamp it (0: no clamp)."""
    B = llr_in.shape[0]
    o = out if out is not None else _empty((B, code.e_tx), torch.float32, llr_in.device)
    _call("lsim_extrinsic", code.handle, _ptr(app, torch.float32, "app"),
          _ptr(llr_in, torch.float32, "llr_in"), llr_max, B, _ptr(o, torch.float32, "out"),
          _stream())
    return o


def demap_q8(m: int, method: int, y, no, scale: float = 2.0, sat: int = 31, out=None):
    B, S = y.shape[0], y.shape[1]
    q = out if out is not None else _empty((B, S * m), torch.int8, y.device)
    _call("lsim_demap_q8", m, method, _ptr(y, torch.float32, "y"), _ptr(no, torch.float32, "no"), B,
          S, scale, sat, _ptr(q, torch.int8, "q"), _stream())
    return q


def quantize(L, scale: float = 2.0, sat: int = 31, out=None):
    q = out if out is not None else torch.empty(L.shape, dtype=torch.int8, device=L.device)
    _call("lsim_quantize", _ptr(L, torch.float32, "llr"), L.numel(), scale, sat,
          _ptr(q, torch.int8, "q"), _stream())
    return q


# --------------------------------------------------------------- decoders

def params(algo: int, iters: int = 20, offset: float = 1.0, alpha: float = 0.75,
           llr_max: float = 20.0, sat: int = 31, threads: int = 0,
           lds_rows: int = 0) -> DecodeParams:
    return DecodeParams(algo, iters, offset, alpha, llr_max, sat, threads, lds_rows)


def decode_launch(code: Code, p: DecodeParams) -> dict:
    """Launch shape of the layered decoder (lsim_decode_launch)."""
    t, g, k, w = _I(), _I(), _I(), _I()
    _call("lsim_decode_launch", code.handle, ctypes.byref(p), ctypes.byref(t), ctypes.byref(g),
          ctypes.byref(k), ctypes.byref(w))
    return {"threads": t.value, "codewords_per_tile": g.value, "lds_rows": k.value,
            "waves_per_simd": w.value}


def decode_workspace(code: Code, p: DecodeParams, B: int) -> int:
    n = ctypes.c_size_t()
    _call("lsim_decode_workspace", code.handle, ctypes.byref(p), B, ctypes.byref(n))
    return n.value


def _work(nbytes, device, work):
    if nbytes == 0:
        return None, 0
    if work is None:
        work = torch.empty(nbytes, dtype=torch.uint8, device=device)
    return work, work.numel() * work.element_size()


def decode(code: Code, llr, p: DecodeParams, want_bits=True, want_app=False, bits=None,
           app=None, work=None):
    """Hard information bits u8[B][k] and/or posteriors L_post f32[B][n_dec]."""
    B = llr.shape[0]
    dt = torch.int8 if p.algo == OMS_I8 else torch.float32
    if want_bits and bits is None:
        bits = _empty((B, code.k), torch.uint8, llr.device)
    if want_app and app is None:
        app = _empty((B, code.n_dec), torch.float32, llr.device)
    work, nbytes = _work(decode_workspace(code, p, B), llr.device, work)
    _call("lsim_decode", code.handle, ctypes.byref(p), _ptr(llr, dt, "llr"), B,
          _ptr(bits, torch.uint8, "bits") if want_bits else None,
          _ptr(app, torch.float32, "app") if want_app else None,
          _ptr(work, None, "work"), nbytes, _stream())
    return bits, app


def decode_noalloc(code: Code, llr, p: DecodeParams, bits, app=None):
    """lsim_decode_noalloc: as decode(), into caller-provided outputs, with the
    layered decoder's state in the library's static device scratch."""
    B = llr.shape[0]
    dt = torch.int8 if p.algo == OMS_I8 else torch.float32
    _call("lsim_decode_noalloc", code.handle, ctypes.byref(p), _ptr(llr, dt, "llr"), B,
          _ptr(bits, torch.uint8, "bits"), _ptr(app, torch.float32, "app"), _stream())
    return bits, app


def decode_state(code: Code, llr, p: DecodeParams, q_in=None, want_q=True, want_r=True):
    """(r, q, L_post) after p.iters rounds, messages in canonical edge order."""
    B = llr.shape[0]
    mt = torch.int8 if p.algo == OMS_I8 else torch.float32
    r = _empty((B, code.E), mt, llr.device) if want_r else None
    q = _empty((B, code.E), mt, llr.device) if (want_q and p.algo != NMS_F32) else None
    app = _empty((B, code.n_dec), torch.float32, llr.device)
    work, nbytes = _work(decode_workspace(code, p, B), llr.device, None)
    _call("lsim_decode_state", code.handle, ctypes.byref(p), _ptr(llr, mt, "llr"), B,
          _ptr(q_in, mt, "q_in"), _ptr(r, mt, "r_out"), _ptr(q, mt, "q_out"),
          _ptr(app, torch.float32, "app"), _ptr(work, None, "work"), nbytes, _stream())
    return r, q, app


def count_errors(ref, hat, bins=None, nbins: int = 1, counts=None):
    B, k = hat.shape
    if counts is None:
        counts = torch.zeros((nbins, 3), dtype=torch.int64, device=hat.device)
    stride = ref.stride(0)
    if ref.stride(1) != 1 or ref.dtype != torch.uint8:
        raise LsimError("ref must be u8 with unit column stride")
    _call("lsim_count_errors", ctypes.c_void_p(ref.data_ptr()), stride, _ptr(hat, torch.uint8, "hat"),
          B, k, _ptr(bins, torch.int32, "bins"), nbins, _ptr(counts, torch.int64, "counts"), _stream())
    return counts


def hard_bits(llr, k: int, out=None):
    """u8[B][k] = [L > 0] of the first k columns of f32 rows."""
    B = llr.shape[0]
    if llr.dtype != torch.float32 or llr.stride(1) != 1:
        raise LsimError("llr must be f32 with unit column stride")
    bits = out if out is not None else _empty((B, k), torch.uint8, llr.device)
    _call("lsim_hard_bits", ctypes.c_void_p(llr.data_ptr()), llr.stride(0), B, k,
          _ptr(bits, torch.uint8, "bits"), _stream())
    return bits


def syndrome(code: Code, hard):
    B = hard.shape[0]
    out = _empty((B,), torch.int32, hard.device)
    if hard.stride(1) != 1 or hard.dtype != torch.uint8:
        raise LsimError("hard decisions must be u8 with unit column stride")
    _call("lsim_syndrome", code.handle, ctypes.c_void_p(hard.data_ptr()), hard.stride(0), B,
          _ptr(out, torch.int32, "unsat"), _stream())
    return out


def ebn0_to_n0(ebn0_db, rate: float, m: int):
    """Noise variance N0 per Eb/N0 in dB (lsim_ebn0_to_n0); a scalar in gives
    a float, an array in gives a float64 array of its shape."""
    import numpy as np
    shape = np.shape(ebn0_db)
    x = np.ascontiguousarray(np.asarray(ebn0_db, dtype=np.float64).reshape(-1))
    out = np.empty_like(x)
    _call("lsim_ebn0_to_n0", x.ctypes.data, x.size, float(rate), int(m), out.ctypes.data)
    return float(out[0]) if shape == () else out.reshape(shape)


PROBE_COPY, PROBE_READ, PROBE_LDS_READ, PROBE_LDS_WRITE, PROBE_FMA, PROBE_EXP2 = range(6)


def probe(kind: int, dst, src=None, nbytes: int = 0, rounds: int = 1, grid: int = 1024) -> int:
    """One peak-rate probe launch (lsim_probe) on the current stream; returns
    the work units it does (bytes or lane operations)."""
    units = _I64()
    _call("lsim_probe", kind, _ptr(src, None, "src") if src is not None else None,
          _ptr(dst, None, "dst"), int(nbytes), int(rounds), int(grid), ctypes.byref(units),
          _stream())
    return units.value


# ----------------------------------------------------------- mixed batches

class MixedPlan:
    """Persistent decode of several codes in one launch (lsim_mixed_plan_*).

    LLRs, bits and posteriors are concatenated by shape in the order of
    ``codes``."""

    def __init__(self, codes, counts, p: DecodeParams, codewords_per_tile=None, threads: int = 0):
        n = len(codes)
        self.codes = list(codes)          # keep the codes alive as long as the plan
        self.counts = [int(x) for x in counts]
        arr = (ctypes.c_void_p * n)(*[c.handle.value for c in codes])
        cnt = (ctypes.c_int64 * n)(*self.counts)
        cpt = None if codewords_per_tile is None else (ctypes.c_int32 * n)(*codewords_per_tile)
        h = ctypes.c_void_p()
        self.p = p
        _call("lsim_mixed_plan_create", ctypes.cast(arr, ctypes.c_void_p),
              ctypes.cast(cnt, ctypes.c_void_p), n, ctypes.byref(p),
              None if cpt is None else ctypes.cast(cpt, ctypes.c_void_p), threads, ctypes.byref(h))
        self._h = h
        nb = ctypes.c_size_t()
        _call("lsim_mixed_workspace", h, ctypes.byref(nb))
        self.work_bytes = nb.value
        self.llr_offsets, self.bits_offsets, self.app_offsets = [], [], []
        lo = bo = ao = 0
        for c, k in zip(codes, self.counts):
            self.llr_offsets.append(lo)
            self.bits_offsets.append(bo)
            self.app_offsets.append(ao)
            lo += k * c.e_tx
            bo += k * c.k
            ao += k * c.n_dec
        self.n_llr, self.n_bits, self.n_app = lo, bo, ao

    def workspace(self, device="cuda"):
        return torch.empty(self.work_bytes, dtype=torch.uint8, device=device)

    def decode(self, llr, bits=None, app=None, work=None, persistent=True):
        if llr.numel() != self.n_llr:
            raise LsimError("concatenated LLRs have the wrong length")
        if bits is not None and bits.numel() != self.n_bits:
            raise LsimError("concatenated bits have the wrong length")
        if app is not None and app.numel() != self.n_app:
            raise LsimError("concatenated posteriors have the wrong length")
        if work is None:
            work = self.workspace(llr.device)
        if work.numel() * work.element_size() < self.work_bytes:
            raise LsimError("workspace too small")
        dt = torch.int8 if self.p.algo == OMS_I8 else torch.float32
        _call("lsim_mixed_decode", self._h, _ptr(llr, dt, "llr"),
              _ptr(bits, torch.uint8, "bits"), _ptr(app, torch.float32, "app"),
              _ptr(work, None, "work"), work.numel(), 1 if persistent else 0, _stream())
        return bits, app

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.lsim_mixed_plan_destroy(h)
            self._h = None


# ----------------------------------------------------- differentiable forms

def wbp_forward(code: Code, w, llr, T: int, llr_max: float = 20.0, ckpt=None, lpost=None,
                want_ckpt: bool = True):
    """Weighted BP forward: L_post f32[B][n_dec] and checkpoints f32[T][B][E]."""
    B = llr.shape[0]
    if lpost is None:
        lpost = _empty((B, code.n_dec), torch.float32, llr.device)
    if want_ckpt and ckpt is None:
        ckpt = _empty((T, B, code.E), torch.float32, llr.device)
    _call("lsim_wbp_forward", code.handle, T, _ptr(w, torch.float32, "w"),
          _ptr(llr, torch.float32, "llr"), B, llr_max, _ptr(ckpt, torch.float32, "ckpt"),
          _ptr(lpost, torch.float32, "lpost"), _stream())
    return lpost, ckpt


def wbp_workspace(code: Code, T: int, B: int) -> int:
    n = ctypes.c_size_t()
    _call("lsim_wbp_workspace", code.handle, T, B, ctypes.byref(n))
    return n.value


def wbp_backward(code: Code, w, llr, ckpt, gpost, T: int, llr_max: float = 20.0, work=None,
                 gllr=None, gw=None):
    """(dLoss/dL_ch f32[B][e_tx], dLoss/dw f32[T][E]) from dLoss/dL_post."""
    B = llr.shape[0]
    if gllr is None:
        gllr = _empty((B, code.e_tx), torch.float32, llr.device)
    if gw is None:
        gw = _empty((T, code.E), torch.float32, llr.device)
    work, nbytes = _work(wbp_workspace(code, T, B), llr.device, work)
    _call("lsim_wbp_backward", code.handle, T, _ptr(w, torch.float32, "w"),
          _ptr(llr, torch.float32, "llr"), _ptr(ckpt, torch.float32, "ckpt"), B, llr_max,
          _ptr(gpost, torch.float32, "gpost"), _ptr(gllr, torch.float32, "gllr"),
          _ptr(gw, torch.float32, "gw"), _ptr(work, None, "work"), nbytes, _stream())
    return gllr, gw


def ndm_forward(params, y, no, out=None):
    B, S = y.shape[0], y.shape[1]
    L = out if out is not None else _empty((B, S * 4), torch.float32, y.device)
    _call("lsim_ndm_forward", _ptr(params, torch.float32, "params"), _ptr(y, torch.float32, "y"),
          _ptr(no, torch.float32, "no"), B, S, _ptr(L, torch.float32, "llr"), _stream())
    return L


def ndm_workspace(B: int, S: int) -> int:
    n = ctypes.c_size_t()
    _call("lsim_ndm_workspace", B, S, ctypes.byref(n))
    return n.value


def points_workspace(code: Code, m: int, B: int) -> int:
    n = ctypes.c_size_t()
    _call("lsim_points_workspace", code.handle, m, B, ctypes.byref(n))
    return n.value


def ndm_backward(params, y, no, gllr, out=None, work=None, gy=None):
    """dLoss/dparams; with ``gy`` (f32[B][S][2], or True to allocate) also
    dLoss/dy, returned as a second value."""
    B, S = y.shape[0], y.shape[1]
    g = out if out is not None else _empty((NDM_PARAMS,), torch.float32, y.device)
    if gy is True:
        gy = _empty((B, S, 2), torch.float32, y.device)
    work, nbytes = _work(ndm_workspace(B, S), y.device, work)
    _call("lsim_ndm_backward", _ptr(params, torch.float32, "params"), _ptr(y, torch.float32, "y"),
          _ptr(no, torch.float32, "no"), _ptr(gllr, torch.float32, "gllr"), B, S,
          _ptr(g, torch.float32, "gparams"),
          _ptr(gy, torch.float32, "gy") if gy is not None else None,
          _ptr(work, None, "work"), nbytes, _stream())
    return (g, gy) if gy is not None else g


def bce_grad(lpost, c, scale: float, want_loss: bool = True, g=None, loss=None, work=None):
    """scale*(sigmoid(L) - c) and scale*sum(softplus(L) - c L); c u8 rows may
    be wider than L (only the first n columns are read)."""
    B, n = lpost.shape
    if g is None:
        g = torch.empty_like(lpost)
    if want_loss and loss is None:
        loss = _empty((1,), torch.float32, lpost.device)
    if c.dtype != torch.uint8 or c.stride(1) != 1:
        raise LsimError("labels must be u8 with unit column stride")
    nb = ctypes.c_size_t()
    _call("lsim_bce_workspace", B, n, ctypes.byref(nb))
    work, nbytes = _work(nb.value if want_loss else 0, lpost.device, work)
    _call("lsim_bce_grad", _ptr(lpost, torch.float32, "lpost"), ctypes.c_void_p(c.data_ptr()),
          c.stride(0), B, n, scale, _ptr(g, torch.float32, "g"),
          _ptr(loss, torch.float32, "loss") if want_loss else None, _ptr(work, None, "work"),
          nbytes, _stream())
    return g, loss


def adam_step(p, g, m, v, step: int, lr: float = 1e-3, beta1: float = 0.9, beta2: float = 0.999,
              eps: float = 1e-8):
    _call("lsim_adam_step", _ptr(p, torch.float32, "p"), _ptr(g, torch.float32, "g"),
          _ptr(m, torch.float32, "m"), _ptr(v, torch.float32, "v"), p.numel(), lr, beta1, beta2,
          eps, step, _stream())


class WBPFunction(torch.autograd.Function):
    """Weighted BP as an autograd function: (L_ch, w) -> L_post, with the
    hand-written adjoint of liblsim and per-round checkpoints."""

    @staticmethod
    def forward(ctx, llr, w, code, T, llr_max):
        lpost, ckpt = wbp_forward(code, w.contiguous(), llr.contiguous(), T, llr_max)
        ctx.save_for_backward(llr, w, ckpt)
        ctx.code, ctx.T, ctx.llr_max = code, T, llr_max
        return lpost

    @staticmethod
    def backward(ctx, gpost):
        llr, w, ckpt = ctx.saved_tensors
        gllr, gw = wbp_backward(ctx.code, w, llr, ckpt, gpost.contiguous(), ctx.T, ctx.llr_max)
        return gllr, gw, None, None, None


class NDMFunction(torch.autograd.Function):
    """Neural demapper as an autograd function: (params, y, N0) -> LLRs."""

    @staticmethod
    def forward(ctx, params, y, no):
        out = ndm_forward(params.contiguous(), y.contiguous(), no.contiguous())
        ctx.save_for_backward(params, y, no)
        return out

    @staticmethod
    def backward(ctx, gllr):
        params, y, no = ctx.saved_tensors
        if ctx.needs_input_grad[1]:
            gp, gy = ndm_backward(params, y, no, gllr.contiguous(), gy=True)
            return gp, gy, None
        return ndm_backward(params, y, no, gllr.contiguous()), None, None


class LinkArgs(ctypes.Structure):
    _fields_ = [("code", _P), ("bits_per_sym", _I), ("demap_method", _I), ("dec", DecodeParams),
                ("q_scale", _F), ("seed", _U64), ("cw0", _I64), ("B", _I64), ("d_no", _P),
                ("d_u", _P), ("d_c", _P), ("d_y", _P), ("d_llr", _P), ("d_bits", _P),
                ("d_work", _P), ("work_bytes", _SZ), ("d_bin", _P), ("nbins", _I),
                ("d_counts", _P)]


class Link:
    """Pre-allocated buffers for lsim_link_run: one call per Monte-Carlo
    batch through source, encoder, mapper + AWGN, demapper, decoder and
    error count.  keep_tx also stores the codewords (c) and channel
    outputs (y); otherwise they stay on chip."""

    def __init__(self, code: Code, m: int, method: int, p: DecodeParams, B: int, no, bins=None,
                 nbins: int = 1, q_scale: float = 2.0, device="cuda", keep_tx: bool = False):
        self.code, self.B = code, B
        self.no = no
        self.u = _empty((B, code.k), torch.uint8, device)
        self.c = _empty((B, code.n_mother), torch.uint8, device) if keep_tx else None
        self.y = _empty((B, code.e_tx // m, 2), torch.float32, device) if keep_tx else None
        self.llr = _empty((B, code.e_tx), torch.int8 if p.algo == OMS_I8 else torch.float32, device)
        self.bits = _empty((B, code.k), torch.uint8, device)
        self.counts = torch.zeros((nbins, 3), dtype=torch.int64, device=device)
        nb = decode_workspace(code, p, B)
        self.work = torch.empty(max(nb, 1), dtype=torch.uint8, device=device)
        self.bins = bins
        self.args = LinkArgs(code.handle, m, method, p, q_scale, 0, 0, B, _ptr(no, torch.float32, "no"),
                             _ptr(self.u), _ptr(self.c), _ptr(self.y), _ptr(self.llr), _ptr(self.bits),
                             _ptr(self.work), nb, _ptr(bins, torch.int32, "bins"), nbins,
                             _ptr(self.counts))

    def run(self, seed: int, cw0: int = 0):
        self.args.seed = seed
        self.args.cw0 = cw0
        _call("lsim_link_run", ctypes.byref(self.args), _stream())

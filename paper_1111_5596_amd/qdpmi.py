"""Python binding of libqdpmi.so (argument marshalling only).

Every ``qdp_*`` function of ``include/qdpmi.h`` is available under the same
name on :data:`lib` (raw ctypes) and through :class:`Context`, which owns one
library context whose pool is a PyTorch ``uint8`` device tensor and whose
stream is PyTorch's current stream.  All arithmetic happens in the library's
HIP kernels; there is no CPU fallback: importing this module without the
built library raises.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqdpmi.so")

# ---- constants mirrored from include/qdpmi.h -----------------------------
QDP_OK = 0
ERRORS = {-1: "QDP_ERR_ARG", -2: "QDP_ERR_TYPE", -3: "QDP_ERR_LATTICE", -4: "QDP_ERR_NOMEM",
          -5: "QDP_ERR_ALIAS", -6: "QDP_ERR_UNSUPPORTED", -7: "QDP_ERR_HIP", -8: "QDP_ERR_STATE"}
TYPES = {"REAL": 0, "COMPLEX": 1, "COLOR_VECTOR": 2, "COLOR_MATRIX": 3, "FERMION": 4,
         "SPIN_MATRIX": 5, "PROPAGATOR": 6, "GAUGE": 7}
PRECS = {"F64": 0, "F32": 1, "F16S": 2}
SUBSETS = {"all": 0, "even": 1, "odd": 2, "timeslice": 3}
SETS = {"all": 0, "parity": 1, "timeslice": 2}
ASSIGN = {"=": 0, "+=": 1, "-=": 2, "*=": 3}
SMEAR_FULL, SMEAR_EVEN_ODD = 0, 1
INIT_NO_AUTOTUNE, INIT_NO_GRAPH, INIT_FLAT_ADDRESSING = 1, 2, 4
RANDOM_SU3, RANDOM_GAUSSIAN = 0, 1
BARYON_PROTON, BARYON_DELTA_PP = 0, 1
OPS = {"field": 0, "gauge": 1, "real_const": 2, "complex_const": 3, "shift": 4, "neg": 5,
       "conj": 6, "adj": 7, "add": 8, "sub": 9, "mul": 10, "gamma_left": 11, "gamma_right": 12,
       "trace": 13, "trace_color": 14, "trace_spin": 15, "real": 16, "imag": 17,
       "local_norm2": 18, "local_inner": 19}
NCOMP = {"REAL": 1, "COMPLEX": 1, "COLOR_VECTOR": 3, "COLOR_MATRIX": 9, "FERMION": 12,
         "SPIN_MATRIX": 16, "PROPAGATOR": 144, "GAUGE": 36}
CANONICAL = {"REAL": (), "COMPLEX": (), "COLOR_VECTOR": (3,), "COLOR_MATRIX": (3, 3),
             "FERMION": (4, 3), "SPIN_MATRIX": (4, 4), "PROPAGATOR": (4, 4, 3, 3)}


class qdp_init_opts(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int32), ("pool_ptr", ctypes.c_void_p),
                ("pool_bytes", ctypes.c_size_t), ("host_spill_bytes", ctypes.c_size_t),
                ("hip_stream", ctypes.c_void_p), ("flags", ctypes.c_uint32)]


class qdp_subset(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("t", ctypes.c_int32)]


class qdp_node(ctypes.Structure):
    _fields_ = [("op", ctypes.c_int32), ("i0", ctypes.c_int32), ("i1", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("field", ctypes.c_uint64),
                ("re", ctypes.c_double), ("im", ctypes.c_double)]


class qdp_expr(ctypes.Structure):
    _fields_ = [("nodes", ctypes.POINTER(qdp_node)), ("n", ctypes.c_int32)]


class qdp_field_info_t(ctypes.Structure):
    _fields_ = [("type", ctypes.c_int32), ("prec", ctypes.c_int32), ("lattice", ctypes.c_uint64),
                ("bytes", ctypes.c_uint64), ("on_device", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class qdp_smear_job(ctypes.Structure):
    _fields_ = [("gauge", ctypes.c_uint64), ("src", ctypes.POINTER(ctypes.c_uint64)),
                ("dst", ctypes.POINTER(ctypes.c_uint64)), ("ncols", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class qdp_cache_stats_t(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in (
        "hits", "misses", "spills", "fills", "bytes_spilled", "bytes_filled", "pool_capacity",
        "pool_limit", "pool_used", "pool_high_water", "host_used", "n_fields", "n_external",
        "external_bytes")]


class qdp_launch_shape(ctypes.Structure):
    _fields_ = [("site_waves", ctypes.c_int32), ("col_groups", ctypes.c_int32),
                ("xcd", ctypes.c_int32), ("waves_per_simd", ctypes.c_int32),
                ("flat", ctypes.c_int32), ("zstack", ctypes.c_int32), ("lds", ctypes.c_int32)]


_c = ctypes
_vp, _u64, _i32, _i64, _dbl, _sz, _u32 = (_c.c_void_p, _c.c_uint64, _c.c_int32, _c.c_int64,
                                          _c.c_double, _c.c_size_t, _c.c_uint32)
_u64p = _c.POINTER(_c.c_uint64)
_dp = _c.POINTER(_c.c_double)

# name -> (restype, argtypes); the complete exported surface of qdpmi.h
SIGNATURES = {
    "qdp_init": (_i32, [_c.POINTER(qdp_init_opts), _c.POINTER(_vp)]),
    "qdp_finalize": (_i32, [_vp]),
    "qdp_lattice_create": (_i32, [_vp, _c.POINTER(_c.c_int32), _u64p]),
    "qdp_field_alloc": (_i32, [_vp, _u64, _i32, _i32, _u64p]),
    "qdp_field_free": (_i32, [_vp, _u64]),
    "qdp_field_host_doubles": (_i32, [_vp, _u64, _c.POINTER(_sz)]),
    "qdp_field_write": (_i32, [_vp, _u64, _dp, _sz]),
    "qdp_field_read": (_i32, [_vp, _u64, _dp, _sz]),
    "qdp_field_info": (_i32, [_vp, _u64, _c.POINTER(qdp_field_info_t)]),
    "qdp_field_read_timeslices": (_i32, [_vp, _u64, _i32, _i32, _dp, _sz]),
    "qdp_eval": (_i32, [_vp, _c.POINTER(qdp_expr), _u64, qdp_subset, _i32]),
    "qdp_shift": (_i32, [_vp, _u64, _u64, _i32, _i32, qdp_subset]),
    "qdp_sum_multi": (_i32, [_vp, _c.POINTER(qdp_expr), _i32, _dp, _sz]),
    "qdp_smear_jacobi": (_i32, [_vp, _u64, _u64p, _i32, _dbl, _i32, _i32, _i32]),
    "qdp_smear_jacobi_to": (_i32, [_vp, _u64, _u64p, _u64p, _i32, _dbl, _i32, _i32, _i32]),
    "qdp_smear_jacobi_batch": (_i32, [_vp, _c.POINTER(qdp_smear_job), _i32, _dbl, _i32]),
    "qdp_hadron_contract": (_i32, [_vp, _u64p, _u64p, _u32, _i32, _i32, _dp]),
    "qdp_hadron_contract_noalloc": (_i32, [_vp, _u64p, _u64p, _u32, _i32, _i32, _vp]),
    "qdp_hadron_contract_mom": (_i32, [_vp, _u64p, _u64p, _u32, _c.POINTER(_c.c_int32), _i32, _i32, _i32,
                                       _dp]),
    "qdp_baryon_contract": (_i32, [_vp, _u64p, _u64p, _i32, _i32, _i32, _i32, _dp]),
    "qdp_cache_stats": (_i32, [_vp, _c.POINTER(qdp_cache_stats_t)]),
    "qdp_cache_evict": (_i32, [_vp, _u64]),
    "qdp_cache_evict_all": (_i32, [_vp]),
    "qdp_set_pool_limit": (_i32, [_vp, _sz]),
    "qdp_fault_alloc_after": (_i32, [_vp, _i64]),
    "qdp_pool_malloc": (_i32, [_vp, _c.c_size_t, _c.POINTER(_vp)]),
    "qdp_pool_free": (_i32, [_vp, _vp]),
    "qdp_sync": (_i32, [_vp]),
    "qdp_last_error": (_c.c_char_p, [_vp]),
    "qdp_fill_random": (_i32, [_vp, _u64, _i32, _u64, _i32, _dbl]),
    "qdp_fill_point": (_i32, [_vp, _u64, _i64, _i32, _i32]),
    "qdp_smear_set_shape": (_i32, [_vp, _c.POINTER(qdp_launch_shape)]),
    "qdp_smear_get_shape": (_i32, [_vp, _c.POINTER(qdp_launch_shape)]),
    "qdp_field_device_ptr": (_i32, [_vp, _u64, _c.POINTER(_vp), _c.POINTER(_u64)]),
}


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    # PyTorch ships its own HIP runtime with the same soname as the system
    # one.  Importing torch first makes libqdpmi.so bind to that runtime, so
    # the process has a single HIP runtime whatever the import order.
    import torch  # noqa: F401

    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built; run `python -m paper_1111_5596_amd.build` "
                           "(there is no CPU fallback)")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = load()


class QdpError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{ERRORS.get(status, status)}: {message}")
        self.status = status


def _u64_array(handles):
    return (ctypes.c_uint64 * len(handles))(*[int(h) for h in handles])


def _propagator(handles, name):
    """The 12 column handles of a propagator as a ctypes array: the C side
    reads exactly 12, so a shorter or longer list is refused here."""
    hs = list(handles)
    if len(hs) != 12:
        raise ValueError(f"{name}: a propagator is 12 column handles, got {len(hs)}")
    return _u64_array(hs)


class Expr:
    """Postfix program for qdp_eval / qdp_sum_multi built from the same tuple
    form the tests use: ('field', handle), ('gauge', handle, mu), ('mul',) ..."""

    def __init__(self, program):
        nodes = (qdp_node * len(program))()
        for i, t in enumerate(program):
            op = t[0]
            n = nodes[i]
            n.op = OPS[op]
            if op == "field":
                n.field = int(t[1])
            elif op == "gauge":
                n.field, n.i0 = int(t[1]), int(t[2])
            elif op == "real_const":
                n.re = float(t[1])
            elif op == "complex_const":
                n.re, n.im = float(t[1]), float(t[2])
            elif op == "shift":
                n.i0, n.i1 = int(t[1]), int(t[2])
            elif op in ("gamma_left", "gamma_right"):
                n.i0 = int(t[1])
        self._nodes = nodes
        self.c = qdp_expr(ctypes.cast(nodes, ctypes.POINTER(qdp_node)), len(program))


def subset(kind="all", t=0):
    if isinstance(kind, tuple):
        kind, t = kind
    return qdp_subset(SUBSETS[kind], int(t))


class Context:
    """One library context on cuda:0 with a PyTorch-owned device pool."""

    def __init__(self, pool_bytes: int = 8 << 30, host_spill_bytes: int = 0, flags: int = 0,
                 device: int = 0):
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("qdpmi needs a HIP device")
        self.device = torch.device("cuda", device)
        pool_bytes = int(pool_bytes) // 256 * 256
        self._pool = torch.empty(pool_bytes, dtype=torch.uint8, device=self.device)
        self._stream = torch.cuda.current_stream(self.device)
        opts = qdp_init_opts(device, ctypes.c_void_p(self._pool.data_ptr()), pool_bytes,
                             int(host_spill_bytes), ctypes.c_void_p(self._stream.cuda_stream),
                             int(flags))
        h = ctypes.c_void_p()
        st = lib.qdp_init(ctypes.byref(opts), ctypes.byref(h))
        if st != QDP_OK:
            raise QdpError(st, "qdp_init failed")
        self.h = h
        self.lattice_dims = {}
        self.field_meta = {}

    # -- plumbing ------------------------------------------------------
    @property
    def stream(self):
        return self._stream

    def check(self, st):
        if st != QDP_OK:
            raise QdpError(st, lib.qdp_last_error(self.h).decode())
        return st

    def close(self):
        if getattr(self, "h", None):
            lib.qdp_finalize(self.h)
            self.h = None
            self._pool = None

    # -- lattices and fields --------------------------------------------
    def lattice(self, dims):
        d = (ctypes.c_int32 * 4)(*[int(x) for x in dims])
        out = ctypes.c_uint64()
        self.check(lib.qdp_lattice_create(self.h, d, ctypes.byref(out)))
        self.lattice_dims[out.value] = tuple(int(x) for x in dims)
        return out.value

    def alloc(self, lat, type_name, prec="F32"):
        out = ctypes.c_uint64()
        self.check(lib.qdp_field_alloc(self.h, lat, TYPES[type_name], PRECS[prec], ctypes.byref(out)))
        self.field_meta[out.value] = (lat, type_name, prec)
        return out.value

    def free(self, f):
        self.check(lib.qdp_field_free(self.h, f))
        self.field_meta.pop(f, None)

    def write(self, f, arr):
        lat, t, _ = self.field_meta[f]
        a = np.asarray(arr)
        if t == "REAL":
            host = np.ascontiguousarray(a.real, dtype=np.float64).reshape(-1)
        else:
            host = np.ascontiguousarray(a, dtype=np.complex128).reshape(-1).view(np.float64)
        self.check(lib.qdp_field_write(self.h, f, host.ctypes.data_as(_dp), host.size))

    def read(self, f):
        lat, t, _ = self.field_meta[f]
        n = ctypes.c_size_t()
        self.check(lib.qdp_field_host_doubles(self.h, f, ctypes.byref(n)))
        host = np.empty(n.value, dtype=np.float64)
        self.check(lib.qdp_field_read(self.h, f, host.ctypes.data_as(_dp), host.size))
        V = int(np.prod(self.lattice_dims[lat]))
        if t == "REAL":
            return host.reshape(V)
        if t == "GAUGE":
            return host.view(np.complex128).reshape(4, V, 3, 3)
        return host.view(np.complex128).reshape((V,) + CANONICAL[t])

    def read_timeslices(self, f, t_begin, t_end):
        """Canonical array of slices t_begin..t_end-1 (a sub-lattice)."""
        lat, t, _ = self.field_meta[f]
        Lx, Ly, Lz, _ = self.lattice_dims[lat]
        Vsub = Lx * Ly * Lz * (t_end - t_begin)
        n = Vsub if t == "REAL" else Vsub * NCOMP[t] * 2
        host = np.empty(n, dtype=np.float64)
        self.check(lib.qdp_field_read_timeslices(self.h, f, t_begin, t_end, host.ctypes.data_as(_dp), n))
        if t == "REAL":
            return host
        if t == "GAUGE":
            return host.view(np.complex128).reshape(4, Vsub, 3, 3)
        return host.view(np.complex128).reshape((Vsub,) + CANONICAL[t])

    def info(self, f):
        out = qdp_field_info_t()
        self.check(lib.qdp_field_info(self.h, f, ctypes.byref(out)))
        return out

    def device_ptr(self, f):
        p, b = ctypes.c_void_p(), ctypes.c_uint64()
        self.check(lib.qdp_field_device_ptr(self.h, f, ctypes.byref(p), ctypes.byref(b)))
        return p.value, b.value

    # -- operations -------------------------------------------------------
    def eval(self, program, dest, sub="all", assign="="):
        e = Expr(program)
        self.check(lib.qdp_eval(self.h, ctypes.byref(e.c), dest, subset(sub), ASSIGN[assign]))

    def shift(self, dest, src, mu, sign, sub="all"):
        self.check(lib.qdp_shift(self.h, dest, src, mu, sign, subset(sub)))

    def sum_multi(self, program, set_kind="all", ncomp=1, nsub=None):
        e = Expr(program)
        n = 2 * ncomp * (nsub or 1)
        out = np.zeros(n, dtype=np.float64)
        self.check(lib.qdp_sum_multi(self.h, ctypes.byref(e.c), SETS[set_kind],
                                     out.ctypes.data_as(_dp), out.size))
        return out.view(np.complex128).reshape(nsub or 1, ncomp)

    def smear(self, gauge, cols, kappa, n_iter, mode=SMEAR_FULL, j_decay=3):
        c = _u64_array(cols)
        self.check(lib.qdp_smear_jacobi(self.h, gauge, c, len(cols), kappa, n_iter, j_decay, mode))

    def smear_to(self, gauge, src, dst, kappa, n_iter, mode=SMEAR_FULL, j_decay=3):
        s, d = _u64_array(src), _u64_array(dst)
        self.check(lib.qdp_smear_jacobi_to(self.h, gauge, s, d, len(src), kappa, n_iter, j_decay, mode))

    def smear_batch(self, jobs, kappa, n_iter):
        """jobs: list of (gauge, src_list, dst_list)."""
        keep = []
        arr = (qdp_smear_job * len(jobs))()
        for i, (g, src, dst) in enumerate(jobs):
            s, d = _u64_array(src), _u64_array(dst)
            keep += [s, d]
            arr[i] = qdp_smear_job(g, ctypes.cast(s, _u64p), ctypes.cast(d, _u64p), len(src), 0)
        self.check(lib.qdp_smear_jacobi_batch(self.h, arr, len(jobs), kappa, n_iter))

    def contract(self, S1, S2, mask=0xFFFF, t0=0, j_decay=3):
        a, b = _propagator(S1, "contract S1"), _propagator(S2, "contract S2")
        lat = self.field_meta[S1[0]][0]
        Lt = self.lattice_dims[lat][3]
        out = np.zeros(16 * Lt * 2, dtype=np.float64)
        self.check(lib.qdp_hadron_contract(self.h, a, b, mask, t0, j_decay,
                                           out.ctypes.data_as(_dp)))
        return out.view(np.complex128).reshape(16, Lt)

    def contract_noalloc(self, S1, S2, out_ptr, mask=0xFFFF, t0=0, j_decay=3):
        """qdp_hadron_contract_noalloc: writes 16 * Lt complex FP64 values
        (the layout of `contract`) to the device address out_ptr, ordered on
        the context stream, without synchronising."""
        a, b = _propagator(S1, "contract_noalloc S1"), _propagator(S2, "contract_noalloc S2")
        self.check(lib.qdp_hadron_contract_noalloc(self.h, a, b, mask, t0, j_decay, _vp(out_ptr)))

    def contract_mom(self, S1, S2, moms, mask=0xFFFF, t0=0, j_decay=3):
        """C_n(p, t), shape (nmom, 16, Lt), for integer momenta `moms`."""
        a, b = _propagator(S1, "contract_mom S1"), _propagator(S2, "contract_mom S2")
        lat = self.field_meta[S1[0]][0]
        Lt = self.lattice_dims[lat][3]
        k = np.ascontiguousarray(np.asarray(moms, dtype=np.int32).reshape(-1, 3))
        out = np.zeros(k.shape[0] * 16 * Lt * 2, dtype=np.float64)
        self.check(lib.qdp_hadron_contract_mom(self.h, a, b, mask,
                                               k.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), k.shape[0],
                                               t0, j_decay, out.ctypes.data_as(_dp)))
        return out.view(np.complex128).reshape(k.shape[0], 16, Lt)

    def nucleon(self, Su, Sd, parity=1, t0=0, j_decay=3):
        """Proton two-point function C(t), shape (Lt,) complex."""
        a, b = _propagator(Su, "nucleon Su"), _propagator(Sd, "nucleon Sd")
        lat = self.field_meta[Su[0]][0]
        Lt = self.lattice_dims[lat][3]
        out = np.zeros(Lt * 2, dtype=np.float64)
        self.check(lib.qdp_baryon_contract(self.h, a, b, BARYON_PROTON, parity, t0,
                                           j_decay, out.ctypes.data_as(_dp)))
        return out.view(np.complex128)

    def delta(self, S, parity=1, t0=0, j_decay=3):
        """Delta++ two-point function C(t) (summed over mu = 1, 2, 3), shape (Lt,) complex."""
        a = _propagator(S, "delta S")
        lat = self.field_meta[S[0]][0]
        Lt = self.lattice_dims[lat][3]
        out = np.zeros(Lt * 2, dtype=np.float64)
        self.check(lib.qdp_baryon_contract(self.h, a, None, BARYON_DELTA_PP, parity, t0, j_decay,
                                           out.ctypes.data_as(_dp)))
        return out.view(np.complex128)

    def fill_random_su3(self, gauge, seed):
        self.check(lib.qdp_fill_random(self.h, gauge, RANDOM_SU3, seed, 0, 1.0))

    def fill_gaussian(self, f, seed, column, scale):
        self.check(lib.qdp_fill_random(self.h, f, RANDOM_GAUSSIAN, seed, column, scale))

    def fill_point(self, f, site, spin, colour):
        self.check(lib.qdp_fill_point(self.h, f, site, spin, colour))

    def cache_stats(self):
        out = qdp_cache_stats_t()
        self.check(lib.qdp_cache_stats(self.h, ctypes.byref(out)))
        return {n: getattr(out, n) for n, _ in qdp_cache_stats_t._fields_}

    def evict(self, f):
        self.check(lib.qdp_cache_evict(self.h, f))

    def evict_all(self):
        self.check(lib.qdp_cache_evict_all(self.h))

    def set_pool_limit(self, nbytes):
        self.check(lib.qdp_set_pool_limit(self.h, nbytes))

    def fault_alloc_after(self, n):
        self.check(lib.qdp_fault_alloc_after(self.h, n))

    def pool_malloc(self, nbytes):
        """Device address (int) of `nbytes` bytes taken from the pool."""
        p = ctypes.c_void_p()
        self.check(lib.qdp_pool_malloc(self.h, nbytes, ctypes.byref(p)))
        return p.value

    def pool_free(self, ptr):
        self.check(lib.qdp_pool_free(self.h, ctypes.c_void_p(ptr)))

    def pool_view(self, ptr, nbytes):
        """A uint8 tensor aliasing `nbytes` of the pool at device address `ptr`
        (the pool is the context's own tensor)."""
        off = ptr - self._pool.data_ptr()
        if off < 0 or off + nbytes > self._pool.numel():
            raise ValueError("address outside the pool")
        return self._pool[off:off + nbytes]

    def set_shape(self, site_waves=0, col_groups=1, xcd=0, waves_per_simd=0, flat=0, zstack=0, lds=0):
        """Force the smearing launch shape (qdp_smear_set_shape; site_waves = 0
        returns to autotuning).  xcd: 0 blocks dealt to the XCDs in turn, 1
        consecutive blocks on one XCD, 2 z-stack groups on one XCD; zstack: the
        waves of a block take tiles one (x, y) plane apart; lds = S: whole-
        lattice F16S updates stage the x/y neighbour window in LDS (blocks of
        2 S waves)."""
        s = qdp_launch_shape(site_waves, col_groups, xcd, waves_per_simd, flat, zstack, lds)
        self.check(lib.qdp_smear_set_shape(self.h, ctypes.byref(s)))

    def get_shape(self):
        """(site_waves, col_groups, xcd, waves_per_simd, flat, zstack, lds) of the last smearing call."""
        s = qdp_launch_shape()
        self.check(lib.qdp_smear_get_shape(self.h, ctypes.byref(s)))
        return (s.site_waves, s.col_groups, s.xcd, s.waves_per_simd, s.flat, s.zstack, s.lds)

    def sync(self):
        self.check(lib.qdp_sync(self.h))

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

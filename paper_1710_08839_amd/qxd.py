"""Python binding of libqxd (ctypes).  Argument marshalling only: every step
of the computation runs in the HIP library.  Device buffers are torch tensors
on the GPU (PyTorch is used for device memory and streams); host inputs are
numpy arrays.  Raises QxdError with the library's message on failure; raises
ImportError if the library has not been built.
"""

import ctypes
import os

import numpy as np

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libqxd.so")

F64, F32, F16S, BF16 = 0, 1, 2, 3
PREC = {"f64": F64, "f32": F32, "f16": F16S, "f16s": F16S, "bf16": BF16}
OP_D, OP_DHAT, OP_HOP, OP_PAULI, OP_OOINV, OP_G5D, OP_DHAT_DAG, OP_NORMAL = 0, 1, 2, 3, 4, 5, 6, 7
NATIVE = 1
EO_GCR, SAP_GCR, DFL_SAP_GCR = 0, 1, 2
STATUS = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "ENOCONV", -4: "EFLOAT", -5: "EDEVICE",
          -6: "EBUSY", -7: "ENOTFOUND"}


class QxdError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Lattice(ctypes.Structure):
    _fields_ = [("dims", ctypes.c_int * 4), ("time_bc", ctypes.c_int), ("cstar", ctypes.c_int),
                ("q_el", ctypes.c_double), ("block", ctypes.c_int * 4), ("cF", ctypes.c_double),
                ("cF_prime", ctypes.c_double)]


class Quark(ctypes.Structure):
    _fields_ = [("kappa", ctypes.c_double), ("q", ctypes.c_double), ("csw", ctypes.c_double),
                ("csw_u1", ctypes.c_double), ("mu", ctypes.c_double), ("theta", ctypes.c_double * 4)]


class Solver(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("tol", ctypes.c_double), ("maxiter", ctypes.c_int),
                ("nkv", ctypes.c_int), ("ncy", ctypes.c_int), ("nmr", ctypes.c_int),
                ("inner_prec", ctypes.c_int), ("inner_tol", ctypes.c_double),
                ("max_outer", ctypes.c_int)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("outer_iters", ctypes.c_int), ("inner_iters", ctypes.c_int),
                ("true_resid", ctypes.c_double), ("seconds", ctypes.c_double)]


class DflParams(ctypes.Structure):
    _fields_ = [("ns", ctypes.c_int), ("ninv", ctypes.c_int), ("ncy", ctypes.c_int), ("nmr", ctypes.c_int),
                ("little_tol", ctypes.c_double), ("little_nkv", ctypes.c_int), ("little_maxiter", ctypes.c_int),
                ("seed", ctypes.c_uint64)]


class Request(ctypes.Structure):
    _fields_ = [("field", ctypes.c_void_p), ("quark", Quark), ("solver", Solver),
                ("eta_dev", ctypes.c_void_p), ("psi_dev", ctypes.c_void_p), ("nrhs", ctypes.c_int)]


class Result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("nrhs", ctypes.c_int), ("latency_s", ctypes.c_double),
                ("queue_s", ctypes.c_double), ("inner_iters", ctypes.c_int),
                ("true_resid", ctypes.c_double)]


# exported symbols and their signatures (also checked by the CPU test-suite)
_VP, _I, _D, _SZ = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t
SIGNATURES = {
    "qxd_abi_version": ([], _I),
    "qxd_last_error": ([], ctypes.c_char_p),
    "qxd_init": ([_I, ctypes.POINTER(_VP)], _I),
    "qxd_finalize": ([_VP], _I),
    "qxd_field_upload": ([_VP, ctypes.POINTER(Lattice), _VP, _VP, ctypes.POINTER(_VP)], _I),
    "qxd_field_release": ([_VP], _I),
    "qxd_field_volume": ([_VP, ctypes.POINTER(ctypes.c_int64)], _I),
    "qxd_spinor_bytes": ([_VP, _I, ctypes.POINTER(_SZ)], _I),
    "qxd_spinor_pack": ([_VP, _I, _VP, _VP, _I, _VP], _I),
    "qxd_spinor_unpack": ([_VP, _I, _VP, _VP, _I, _VP], _I),
    "qxd_dirac_apply": ([_VP, ctypes.POINTER(Quark), _I, _I, _I, _VP, _VP, _I, ctypes.c_uint, _VP], _I),
    "qxd_dirac_apply_noalloc": ([_VP, ctypes.POINTER(Quark), _I, _I, _I, _VP, _VP, _I, ctypes.c_uint, _VP],
                                _I),
    "qxd_solve": ([_VP, ctypes.POINTER(Quark), _I, ctypes.POINTER(Solver), _VP, _VP, _I, _I,
                   ctypes.POINTER(SolveInfo), _VP], _I),
    "qxd_sap_apply": ([_VP, ctypes.POINTER(Quark), _I, _I, _I, _VP, _VP, _I, _VP], _I),
    "qxd_multishift_solve": ([_VP, ctypes.POINTER(Quark), _VP, _I, _D, _I, _VP, _VP, ctypes.POINTER(SolveInfo),
                              _VP], _I),
    "qxd_rational_apply": ([_VP, ctypes.POINTER(Quark), _D, _VP, _VP, _I, _D, _I, _VP, _VP,
                            ctypes.POINTER(SolveInfo), _VP], _I),
    "qxd_dfl_setup": ([_VP, ctypes.POINTER(Quark), ctypes.POINTER(DflParams), _VP, _VP], _I),
    "qxd_serve_start": ([_VP, _SZ, _I], _I),
    "qxd_serve_submit": ([_VP, ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_uint64)], _I),
    "qxd_serve_poll": ([_VP, ctypes.c_uint64, ctypes.POINTER(Result)], _I),
    "qxd_serve_stop": ([_VP], _I),
    # testing hooks (include/qxd_debug.h)
    "qxd_debug_set_dirac_variant": ([_I], _I),
    "qxd_debug_set_step_graphs": ([_I], _I),
    "qxd_debug_set_gs_passes": ([_I], _I),
    "qxd_debug_fail_steps": ([_I], _I),
    "qxd_debug_serve_charges": ([_VP, ctypes.POINTER(ctypes.c_size_t)], _I),
    "qxd_debug_sap_pair_pass": ([_VP, ctypes.POINTER(Quark), _I, _I, _I, _I, ctypes.POINTER(ctypes.c_float), _VP],
                                _I),
    "qxd_debug_stream": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, _I, ctypes.c_void_p], _I),
    "qxd_debug_step_graph_counts": ([ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)], _I),
    "qxd_debug_get_dirac_variant": ([_VP, _I, ctypes.POINTER(_I)], _I),
    "qxd_debug_dfl_basis": ([_VP, ctypes.POINTER(Quark), _I, _VP, _VP], _I),
    "qxd_debug_dfl_little": ([_VP, ctypes.POINTER(Quark), ctypes.POINTER(_I), ctypes.POINTER(_I), _VP, _VP], _I),
    "qxd_debug_dfl_precond": ([_VP, ctypes.POINTER(Quark), _D, _I, _I, _VP, _VP, _VP], _I),
    "qxd_debug_dfl_stats": ([_VP, ctypes.POINTER(Quark), ctypes.POINTER(ctypes.c_int64)], _I),
}

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise ImportError(f"libqxd.so not built ({_LIB_PATH}); run python -m paper_1710_08839_amd.build")
        # PyTorch carries its own HIP runtime (same soname as the system one).
        # Load it first so that libqxd binds to the same runtime instance and
        # both share one device context, allocator view and stream namespace.
        import torch  # noqa: F401
        _lib = ctypes.CDLL(_LIB_PATH)
        for name, (args, res) in SIGNATURES.items():
            fn = getattr(_lib, name)
            fn.argtypes = args
            fn.restype = res
    return _lib


def _check(status):
    if status != 0:
        raise QxdError(status, lib().qxd_last_error().decode())


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    return getattr(stream, "cuda_stream", stream)


def _ptr(t):
    return t.data_ptr() if hasattr(t, "data_ptr") else int(t)


def set_dirac_variant(choice=0):
    """Force a Dirac kernel variant (hop group 1/2/4/8, +16 for LDS staging,
    +32 for non-temporal Pauli/output streams, +64 for mirror-fused link
    reads, +128 for wavefront-uniform addressing on 4^4 blocks, the last three
    with LDS staging); 0 returns to the autotuner.  A testing hook."""
    _check(lib().qxd_debug_set_dirac_variant(int(choice)))


def set_step_graphs(enable=True):
    """Replay batched SAP-GCR steps from captured HIP graphs (default) or
    issue every launch directly.  A testing hook."""
    _check(lib().qxd_debug_set_step_graphs(1 if enable else 0))


def set_gs_passes(passes=1):
    """Classical Gram-Schmidt passes (1, or 2 with one re-orthogonalisation)
    per step of batched SAP-GCR solvers created after the call.  A
    measurement hook."""
    _check(lib().qxd_debug_set_gs_passes(int(passes)))


def last_error():
    """The calling thread's last error message of the library."""
    m = lib().qxd_last_error()
    return m.decode() if m else ""


def fail_steps(n):
    """Make the next n batched SAP-GCR steps fail before any device work
    (0 cancels).  A testing hook for the error paths."""
    _check(lib().qxd_debug_fail_steps(int(n)))


def stream_probe(src, dst, dst_bytes, reads_per_write, stream=None):
    """dst = xor of reads_per_write planes of src (device tensors, 16-byte
    aligned), with the library's streaming kernel.  A measurement hook."""
    _check(lib().qxd_debug_stream(_ptr(src), _ptr(dst), int(dst_bytes), int(reads_per_write),
                                  _stream(stream)))


def step_graph_counts():
    """(captures, launches) of batched-step HIP graphs so far in this
    process.  A testing hook."""
    c, r = ctypes.c_int64(0), ctypes.c_int64(0)
    _check(lib().qxd_debug_step_graph_counts(ctypes.byref(c), ctypes.byref(r)))
    return c.value, r.value


def quark(kappa, q=0.0, csw=0.0, csw_u1=1.0, mu=0.0, theta=(0.0, 0.0, 0.0, 0.0)):
    """Quark parameters: hopping parameter, charge, clover coefficients,
    twisted mass of the even-odd normal operators, fermion boundary phases."""
    return Quark(kappa, q, csw, csw_u1, mu, (ctypes.c_double * 4)(*theta))


def solver(kind=SAP_GCR, tol=1e-10, maxiter=0, nkv=0, ncy=0, nmr=0, inner_prec=F32, inner_tol=0.0,
           max_outer=0):
    return Solver(kind, tol, maxiter, nkv, ncy, nmr, inner_prec, inner_tol, max_outer)


class Context:
    def __init__(self, device=0):
        self.h = ctypes.c_void_p()
        _check(lib().qxd_init(device, ctypes.byref(self.h)))

    def close(self):
        if self.h:
            _check(lib().qxd_finalize(self.h))
            self.h = ctypes.c_void_p()

    # serving
    def serve_start(self, budget_bytes=0, max_active=0):
        _check(lib().qxd_serve_start(self.h, budget_bytes, max_active))

    def serve_submit(self, field, q, s, eta, psi, nrhs):
        req = Request(field.h, q, s, _ptr(eta), _ptr(psi), nrhs)
        t = ctypes.c_uint64()
        _check(lib().qxd_serve_submit(self.h, ctypes.byref(req), ctypes.byref(t)))
        return t.value

    def serve_poll(self, ticket):
        """None while pending, else the Result."""
        r = Result()
        st = lib().qxd_serve_poll(self.h, ticket, ctypes.byref(r))
        if st == -6:
            return None
        _check(st)
        return r

    def serve_stop(self):
        _check(lib().qxd_serve_stop(self.h))

    def serve_charges(self):
        """The serve loop's memory accounting (a testing hook): operator bytes
        admitted requests have still to build, operator bytes the fields have
        built since serving saw them, solver slot bytes, and the budget."""
        out = (ctypes.c_size_t * 4)()
        _check(lib().qxd_debug_serve_charges(self.h, out))
        return {"op_pending": out[0], "op_resident": out[1], "slots": out[2], "budget": out[3]}


class Field:
    """A resident gauge field (physical-lattice U and optional A, host numpy)."""

    def __init__(self, ctx, dims, u, a=None, cstar=0, time_bc=0, q_el=1.0 / 6.0, block=(4, 4, 4, 4), cF=1.0,
                 cF_prime=1.0):
        self.ctx = ctx
        self.lat = Lattice((ctypes.c_int * 4)(*dims), time_bc, cstar, q_el, (ctypes.c_int * 4)(*block), cF,
                           cF_prime)
        u = np.ascontiguousarray(u, dtype=np.complex128)
        a_ptr = None
        if a is not None:
            a = np.ascontiguousarray(a, dtype=np.float64)
            a_ptr = a.ctypes.data
        self.h = ctypes.c_void_p()
        _check(lib().qxd_field_upload(ctx.h, ctypes.byref(self.lat), u.ctypes.data, a_ptr, ctypes.byref(self.h)))
        v = ctypes.c_int64()
        _check(lib().qxd_field_volume(self.h, ctypes.byref(v)))
        self.volume = v.value

    def release(self):
        if self.h:
            _check(lib().qxd_field_release(self.h))
            self.h = ctypes.c_void_p()

    def spinor_bytes(self, prec):
        n = ctypes.c_size_t()
        _check(lib().qxd_spinor_bytes(self.h, prec, ctypes.byref(n)))
        return n.value

    def pack(self, prec, api, native, nrhs=1, stream=None):
        _check(lib().qxd_spinor_pack(self.h, prec, _ptr(api), _ptr(native), nrhs, _stream(stream)))

    def unpack(self, prec, native, api, nrhs=1, stream=None):
        _check(lib().qxd_spinor_unpack(self.h, prec, _ptr(native), _ptr(api), nrhs, _stream(stream)))

    def dirac_variant(self, prec):
        """Kernel variant the autotuner chose for D in precision prec (0 if
        D has not been applied yet): hop group + 16 (LDS staging) + 32
        (non-temporal streams)."""
        c = ctypes.c_int(0)
        _check(lib().qxd_debug_get_dirac_variant(self.h, int(prec), ctypes.byref(c)))
        return c.value

    def apply(self, quarks, op, prec, x, y, nrhs=1, native=False, stream=None):
        qs = quarks if isinstance(quarks, (list, tuple)) else [quarks]
        arr = (Quark * len(qs))(*qs)
        _check(lib().qxd_dirac_apply(self.h, arr, len(qs), op, prec, _ptr(x), _ptr(y), nrhs,
                                     NATIVE if native else 0, _stream(stream)))

    def apply_noalloc(self, quarks, op, prec, x, y, nrhs=1, native=False, stream=None):
        """As apply, through the allocation-free entry point (the operators
        must already be built in precision prec)."""
        qs = quarks if isinstance(quarks, (list, tuple)) else [quarks]
        arr = (Quark * len(qs))(*qs)
        _check(lib().qxd_dirac_apply_noalloc(self.h, arr, len(qs), op, prec, _ptr(x), _ptr(y), nrhs,
                                             NATIVE if native else 0, _stream(stream)))

    def solve(self, quarks, s, eta, psi, nrhs=1, use_guess=False, stream=None, check=True):
        qs = quarks if isinstance(quarks, (list, tuple)) else [quarks]
        arr = (Quark * len(qs))(*qs)
        info = (SolveInfo * nrhs)()
        st = lib().qxd_solve(self.h, arr, len(qs), ctypes.byref(s), _ptr(eta), _ptr(psi), nrhs,
                             int(use_guess), info, _stream(stream))
        if check and st not in (0,):
            _check(st)
        return st, list(info)

    def multishift(self, q, shifts, eta, psi, tol=1e-10, maxiter=0, stream=None, check=True):
        """(D^dag D^ + mu^2 + shifts[j]) psi[j] = eta on the even sites; psi
        holds len(shifts) API-layout spinors.  Returns (status, infos)."""
        sh = np.ascontiguousarray(shifts, dtype=np.float64)
        info = (SolveInfo * len(sh))()
        st = lib().qxd_multishift_solve(self.h, ctypes.byref(q), sh.ctypes.data, len(sh), float(tol), int(maxiter),
                                        _ptr(eta), _ptr(psi), info, _stream(stream))
        if check and st != 0:
            _check(st)
        return st, list(info)

    def rational(self, q, A, nu, mu, eta, out, tol=1e-10, maxiter=0, stream=None, check=True):
        """out = A prod_j (X + nu_j^2) / (X + mu_j^2) eta, X = D^dag D^ +
        q.mu^2, on the even sites.  Returns (status, infos per pole)."""
        nu = np.ascontiguousarray(nu, dtype=np.float64)
        mu = np.ascontiguousarray(mu, dtype=np.float64)
        info = (SolveInfo * len(mu))()
        st = lib().qxd_rational_apply(self.h, ctypes.byref(q), float(A), nu.ctypes.data, mu.ctypes.data, len(mu),
                                      float(tol), int(maxiter), _ptr(eta), _ptr(out), info, _stream(stream))
        if check and st != 0:
            _check(st)
        return st, list(info)

    def dfl_setup(self, q, ns=0, ninv=0, ncy=0, nmr=0, little_tol=0.0, little_nkv=0, little_maxiter=0, seed=0,
                  init=None, stream=None):
        """Build the local deflation subspace and little operator of quark q
        (start fields: init, ns API-layout FP64 spinors on the device, or
        random from seed)."""
        p = DflParams(ns, ninv, ncy, nmr, little_tol, little_nkv, little_maxiter, seed)
        _check(lib().qxd_dfl_setup(self.h, ctypes.byref(q), ctypes.byref(p), _ptr(init) if init is not None else None,
                                   _stream(stream)))

    def dfl_basis(self, q, k, out, stream=None):
        """Basis field k of the deflation subspace into the API-layout FP64
        spinor out (a testing hook)."""
        _check(lib().qxd_debug_dfl_basis(self.h, ctypes.byref(q), int(k), _ptr(out), _stream(stream)))

    def dfl_little(self, q):
        """The little operator as a complex array [nblocks, 9, ns, ns] and the
        neighbour table [nblocks, 9] (a testing hook)."""
        ns, nb = _I(0), _I(0)
        _check(lib().qxd_debug_dfl_little(self.h, ctypes.byref(q), ctypes.byref(ns), ctypes.byref(nb), None, None))
        a = np.empty((nb.value, 9, ns.value, ns.value), dtype=np.complex128)
        nbr = np.empty((nb.value, 9), dtype=np.int32)
        _check(lib().qxd_debug_dfl_little(self.h, ctypes.byref(q), ctypes.byref(ns), ctypes.byref(nb),
                                          a.ctypes.data, nbr.ctypes.data))
        return a, nbr

    def dfl_stats(self, q):
        """(preconditioner applications, little GCR iterations, most in one
        little solve) since the last call; a measurement hook."""
        out = (ctypes.c_int64 * 3)()
        _check(lib().qxd_debug_dfl_stats(self.h, ctypes.byref(q), out))
        return tuple(out)

    def dfl_precond(self, q, x, y, little_tol=0.0, ncy=4, nmr=4, stream=None):
        """y = M_dfl x (API-layout FP64 spinors; a testing hook)."""
        _check(lib().qxd_debug_dfl_precond(self.h, ctypes.byref(q), float(little_tol), int(ncy), int(nmr), _ptr(x),
                                           _ptr(y), _stream(stream)))

    def sap_pair_pass_ms(self, q, prec, nmr=4, npair=1, reps=20, stream=None):
        """Average time (ms) of one colour pass of the paired SAP block
        solver on synthetic vectors.  A measurement hook."""
        t = ctypes.c_float(0)
        _check(lib().qxd_debug_sap_pair_pass(self.h, ctypes.byref(q), int(prec), int(nmr), int(npair), int(reps),
                                             ctypes.byref(t), _stream(stream)))
        return t.value

    def sap_apply(self, q, prec, ncy, nmr, x, y, nrhs=1, stream=None):
        _check(lib().qxd_sap_apply(self.h, ctypes.byref(q), prec, ncy, nmr, _ptr(x), _ptr(y), nrhs,
                                   _stream(stream)))

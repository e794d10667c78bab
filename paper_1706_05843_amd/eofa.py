"""ctypes binding of libeofa.so (include/eofa.h).

Argument marshalling only: every step of the solve runs in the HIP library.
Fields are torch tensors on the GPU (complex128 canonical layout, or uint8
buffers holding packed half-fields); their data pointers and torch's current
HIP stream are handed to the C entry points of the same names.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libeofa.so")

EOFA_OK = 0
EOFA_ERR_INVALID = -1
EOFA_ERR_NOT_CONVERGED = -2
EOFA_ERR_BREAKDOWN = -3
EOFA_ERR_HIP = -4
EOFA_ERR_OOM = -5

FP64, FP32, FP16S = 0, 1, 2

MAT_NAMES = ["mee", "mee_inv", "mee_t", "mee_inv_t", "mee_inv_t_dt_t", "neg_dt_t", "dt_t", "dt", "dt_inv",
             "dee", "dee_inv", "dee_t", "dee_inv_t"]


class Action(ctypes.Structure):
    _fields_ = [("dims", ctypes.c_int32 * 4), ("Ls", ctypes.c_int32), ("M5", ctypes.c_double),
                ("b5", ctypes.c_double), ("c5", ctypes.c_double), ("bc", ctypes.c_int32 * 4)]


class System(ctypes.Structure):
    _fields_ = [("m_op", ctypes.c_double), ("m_a", ctypes.c_double), ("m_b", ctypes.c_double),
                ("beta", ctypes.c_double), ("chi", ctypes.c_int32)]


class SolverParams(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_iter", ctypes.c_int32), ("max_outer", ctypes.c_int32),
                ("inner_prec", ctypes.c_int32), ("inner_tol", ctypes.c_double),
                ("fixed_iters", ctypes.c_int32), ("check_every", ctypes.c_int32),
                ("profile", ctypes.c_int32), ("use_graph", ctypes.c_int32), ("rhs_block", ctypes.c_int32),
                ("waves", ctypes.c_int32), ("precond", ctypes.c_int32), ("fcg_window", ctypes.c_int32),
                ("net", ctypes.c_void_p), ("use_guess", ctypes.c_int32), ("form", ctypes.c_int32),
                ("keep_direction", ctypes.c_int32), ("ring_slots", ctypes.c_int32)]


class SolverStats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("outer_iters", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("status", ctypes.c_int32), ("true_resid", ctypes.c_double), ("seconds", ctypes.c_double),
                ("hop_ms", ctypes.c_double * 4), ("hop_timed", ctypes.c_int32), ("waves", ctypes.c_int32),
                ("rhs_block", ctypes.c_int32), ("fell_back", ctypes.c_int32)]

    def as_dict(self):
        return dict(iters=self.iters, outer_iters=self.outer_iters, converged=self.converged,
                    status=self.status, true_resid=self.true_resid, seconds=self.seconds,
                    hop_ms=list(self.hop_ms), hop_timed=self.hop_timed, waves=self.waves,
                    rhs_block=self.rhs_block, fell_back=self.fell_back)


_LIB = None
_P = ctypes.c_void_p
_I = ctypes.c_int32


def lib():
    """Load libeofa.so; raises if it is missing (there is no fallback)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1706_05843_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    sig = {
        "eofa_create": ([ctypes.POINTER(Action), _P, _P, ctypes.POINTER(_P)], _I),
        "eofa_destroy": ([_P], _I),
        "eofa_last_error": ([], ctypes.c_char_p),
        "eofa_packed_bytes": ([_P, _I, _I], ctypes.c_size_t),
        "eofa_pack": ([_P, _P, _P, _I, _I, _I, _I, _P], _I),
        "eofa_unpack": ([_P, _P, _P, _I, _I, _I, _P], _I),
        "eofa_dslash": ([_P, ctypes.POINTER(System), _P, _P, _I, _I, _I, _I, _P], _I),
        "eofa_mooee": ([_P, ctypes.POINTER(System), _P, _P, _I, _I, _I, _P], _I),
        "eofa_mooee_inv": ([_P, ctypes.POINTER(System), _P, _P, _I, _I, _I, _P], _I),
        "eofa_cg_solve": ([_P, ctypes.POINTER(System), _P, _P, _I, ctypes.POINTER(SolverParams),
                           ctypes.POINTER(SolverStats), _P], _I),
        "eofa_cg_solve_noalloc": ([_P, ctypes.POINTER(System), _P, _P, _I, ctypes.POINTER(SolverParams),
                                   ctypes.POINTER(SolverStats), _P], _I),
        "eofa_heatbath_solve": ([_P, ctypes.c_double, ctypes.c_double, _I, ctypes.POINTER(ctypes.c_double),
                                 ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double), _P, _P,
                                 ctypes.POINTER(SolverParams), ctypes.POINTER(SolverStats), _P], _I),
        "eofa_heatbath_poles": ([_P, ctypes.c_double, ctypes.c_double, _I, ctypes.POINTER(ctypes.c_double),
                                 ctypes.POINTER(ctypes.c_double), _P, _P, ctypes.POINTER(SolverParams),
                                 ctypes.POINTER(SolverStats), _P], _I),
        "eofa_forecast": ([_P, ctypes.POINTER(System), _P, _P, _I, _P, _P], _I),
        "eofa_fifth_matrix": ([ctypes.POINTER(Action), ctypes.POINTER(System), _I,
                               ctypes.POINTER(ctypes.c_double)], _I),
        "eofa_dhop_derivative": ([_P, _P, _P, _P, _P], _I),
        "eofa_force": ([_P, ctypes.c_double, ctypes.c_double, _P, _P, ctypes.POINTER(SolverParams),
                        ctypes.POINTER(SolverStats), _P], _I),
        "eofa_cg_pairs": ([_P, ctypes.POINTER(System), _P, _I, _I, _I, ctypes.c_double, _I, _P, _P,
                           ctypes.POINTER(_I), ctypes.POINTER(_I), _P], _I),
        "eofa_net_create": ([_P, _I, ctypes.POINTER(_I), ctypes.c_uint64, ctypes.c_double, ctypes.POINTER(_P)], _I),
        "eofa_net_destroy": ([_P], _I),
        "eofa_net_num_weights": ([_P], ctypes.c_size_t),
        "eofa_net_get_weights": ([_P, ctypes.POINTER(ctypes.c_double)], _I),
        "eofa_net_set_weights": ([_P, ctypes.POINTER(ctypes.c_double)], _I),
        "eofa_net_apply": ([_P, _P, _P, _P, _P], _I),
        "eofa_net_loss_grad": ([_P, _P, ctypes.POINTER(System), _P, _P, _I, ctypes.POINTER(ctypes.c_double),
                                ctypes.POINTER(ctypes.c_double), _P], _I),
        "eofa_net_train": ([_P, _P, ctypes.POINTER(System), _P, _P, _I, _I, _I, ctypes.c_double,
                            ctypes.POINTER(ctypes.c_double), _P], _I),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _LIB = L
    return L


class EofaError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"eofa error {code}: {msg}")
        self.code = code


def _check(rc):
    if rc != EOFA_OK:
        raise EofaError(rc, lib().eofa_last_error().decode())
    return rc


def make_action(dims, Ls, M5, b5, c5, bc=(1, 1, 1, -1)):
    a = Action()
    for k in range(4):
        a.dims[k] = int(dims[k])
        a.bc[k] = int(bc[k])
    a.Ls, a.M5, a.b5, a.c5 = int(Ls), float(M5), float(b5), float(c5)
    return a


def make_systems(systems):
    """systems: list of (m_op, m_a, m_b, beta, chi) tuples or objects with those attributes."""
    arr = (System * len(systems))()
    for k, s in enumerate(systems):
        if isinstance(s, tuple):
            m_op, m_a, m_b, beta, chi = s
        else:
            m_op, m_a, m_b, beta, chi = s.m_op, s.m_a, s.m_b, s.beta, s.chi
        arr[k].m_op, arr[k].m_a, arr[k].m_b, arr[k].beta, arr[k].chi = m_op, m_a, m_b, beta, int(chi)
    return arr


def make_params(tol=1e-10, max_iter=100000, max_outer=20, inner_prec=FP64, inner_tol=0.0,
                fixed_iters=0, check_every=16, profile=0, use_graph=0, rhs_block=0, waves=0,
                precond=0, net=None, fcg_window=0, use_guess=0, form=0, keep_direction=0, ring_slots=0):
    """Solver parameters; ``net`` (a Net, or None for the identity) is used when precond = 1;
    ``form`` 0 is the Cayley form, 1 the dense comparison form."""
    p = SolverParams()
    p.tol, p.max_iter, p.max_outer, p.inner_prec = tol, max_iter, max_outer, inner_prec
    p.inner_tol, p.fixed_iters, p.check_every, p.profile = inner_tol, fixed_iters, check_every, profile
    p.use_graph, p.rhs_block, p.waves = use_graph, rhs_block, waves
    p.precond, p.fcg_window, p.use_guess, p.form = precond, fcg_window, use_guess, form
    p.keep_direction, p.ring_slots = keep_direction, ring_slots
    p.net = net._h.value if net is not None else None
    p._net_ref = net  # keeps the network alive as long as the parameters
    return p


def eofa_fifth_matrix(action, system, mat):
    """Host-only: the [2][Ls][Ls] fifth-dimension matrix ``mat`` (name or index) the library builds."""
    if isinstance(mat, str):
        mat = MAT_NAMES.index(mat)
    Ls = action.Ls
    out = (ctypes.c_double * (2 * Ls * Ls))()
    _check(lib().eofa_fifth_matrix(ctypes.byref(action), make_systems([system]), mat, out))
    return np.frombuffer(out, dtype=np.float64).reshape(2, Ls, Ls).copy()


def _stream(stream):
    if stream is not None:
        return ctypes.c_void_p(stream)
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class Context:
    """An eofa_ctx: the action and the packed gauge field on the current GPU."""

    def __init__(self, action, gauge, stream=None):
        import torch
        assert gauge.is_cuda and gauge.dtype == torch.complex128 and gauge.is_contiguous()
        self.action = action
        self.dims = tuple(action.dims)
        self.Ls = action.Ls
        self.gparity = action.bc[0] == 2
        self._h = ctypes.c_void_p()
        _check(lib().eofa_create(ctypes.byref(action), ctypes.c_void_p(gauge.data_ptr()), _stream(stream),
                                 ctypes.byref(self._h)))

    def close(self):
        if self._h:
            lib().eofa_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # --- buffers -----------------------------------------------------------
    def packed_bytes(self, prec, nrhs=1):
        return int(lib().eofa_packed_bytes(self._h, prec, nrhs))

    def new_packed(self, prec, nrhs=1):
        import torch
        return torch.empty(self.packed_bytes(prec, nrhs), dtype=torch.uint8, device="cuda")

    def full_shape(self, nrhs=1):
        """Canonical fermion shape; with G-parity in x the flavour axis sits between y and x."""
        lx, ly, lz, lt = self.dims
        if self.gparity:
            return (nrhs, self.Ls, lt, lz, ly, 2, lx, 4, 3)
        return (nrhs, self.Ls, lt, lz, ly, lx, 4, 3)

    # --- entry points ------------------------------------------------------
    def eofa_pack(self, full, packed, parity, prec, nrhs=1, g5r5=0, stream=None):
        _check(lib().eofa_pack(self._h, _p(full), _p(packed), parity, prec, nrhs, g5r5, _stream(stream)))

    def eofa_unpack(self, packed, full, parity, prec, nrhs=1, stream=None):
        _check(lib().eofa_unpack(self._h, _p(packed), _p(full), parity, prec, nrhs, _stream(stream)))

    def eofa_dslash(self, systems, inp, out, out_parity, dagger=0, prec=FP64, nrhs=1, stream=None):
        _check(lib().eofa_dslash(self._h, make_systems(systems), _p(inp), _p(out), out_parity, dagger, prec,
                                 nrhs, _stream(stream)))

    def eofa_mooee(self, systems, inp, out, dagger=0, prec=FP64, nrhs=1, stream=None):
        _check(lib().eofa_mooee(self._h, make_systems(systems), _p(inp), _p(out), dagger, prec, nrhs,
                                _stream(stream)))

    def eofa_mooee_inv(self, systems, inp, out, dagger=0, prec=FP64, nrhs=1, stream=None):
        _check(lib().eofa_mooee_inv(self._h, make_systems(systems), _p(inp), _p(out), dagger, prec, nrhs,
                                    _stream(stream)))

    def eofa_cg_solve(self, systems, phi, psi, params, stream=None, raise_on=("invalid", "hip", "oom")):
        n = len(systems)
        stats = (SolverStats * n)()
        rc = lib().eofa_cg_solve(self._h, make_systems(systems), _p(phi), _p(psi), n, ctypes.byref(params),
                                 stats, _stream(stream))
        if rc in (EOFA_ERR_INVALID, EOFA_ERR_HIP, EOFA_ERR_OOM):
            _check(rc)
        return rc, [s.as_dict() for s in stats]

    def eofa_cg_solve_noalloc(self, systems, phi, psi, params, stream=None):
        """eofa_cg_solve without device allocation (workspace in the library's scratch array)."""
        n = len(systems)
        stats = (SolverStats * n)()
        rc = lib().eofa_cg_solve_noalloc(self._h, make_systems(systems), _p(phi), _p(psi), n,
                                         ctypes.byref(params), stats, _stream(stream))
        if rc in (EOFA_ERR_INVALID, EOFA_ERR_HIP, EOFA_ERR_OOM):
            _check(rc)
        return rc, [s.as_dict() for s in stats]

    def eofa_heatbath_solve(self, m1, m2, alpha, beta, eta, phi, params, pole_tol=None, stream=None):
        npol = len(beta)
        assert len(alpha) == npol + 1
        a = (ctypes.c_double * (npol + 1))(*alpha)
        b = (ctypes.c_double * npol)(*beta)
        pt = None
        if pole_tol is not None:
            assert len(pole_tol) == 2 * npol
            pt = (ctypes.c_double * (2 * npol))(*pole_tol)
        stats = (SolverStats * (2 * npol))()
        rc = lib().eofa_heatbath_solve(self._h, m1, m2, npol, a, b, pt, _p(eta), _p(phi), ctypes.byref(params),
                                       stats, _stream(stream))
        if rc in (EOFA_ERR_INVALID, EOFA_ERR_HIP, EOFA_ERR_OOM):
            _check(rc)
        return rc, [s.as_dict() for s in stats]

    def eofa_heatbath_poles(self, m1, m2, beta, eta, sol, params, pole_tol=None, stream=None):
        """The 2 len(beta) pole solutions (LH then RH) into sol (canonical, [2 N_p, ...])."""
        npol = len(beta)
        b = (ctypes.c_double * npol)(*beta)
        pt = None
        if pole_tol is not None:
            assert len(pole_tol) == 2 * npol
            pt = (ctypes.c_double * (2 * npol))(*pole_tol)
        stats = (SolverStats * (2 * npol))()
        rc = lib().eofa_heatbath_poles(self._h, m1, m2, npol, b, pt, _p(eta), _p(sol), ctypes.byref(params),
                                       stats, _stream(stream))
        if rc in (EOFA_ERR_INVALID, EOFA_ERR_HIP, EOFA_ERR_OOM):
            _check(rc)
        return rc, [s.as_dict() for s in stats]

    def eofa_forecast(self, system, rhs, prev, n_prev, guess, stream=None):
        """Chronological guess for ``system`` over n_prev canonical fields ``prev``."""
        _check(lib().eofa_forecast(self._h, make_systems([system]), _p(rhs), _p(prev), n_prev, _p(guess),
                                   _stream(stream)))

    def eofa_dhop_derivative(self, a, b, y, stream=None):
        _check(lib().eofa_dhop_derivative(self._h, _p(a), _p(b), _p(y), _stream(stream)))

    def eofa_force(self, m1, m2, phi, force, params, stream=None):
        stats = (SolverStats * 2)()
        rc = lib().eofa_force(self._h, m1, m2, _p(phi), _p(force), ctypes.byref(params), stats, _stream(stream))
        if rc in (EOFA_ERR_INVALID, EOFA_ERR_HIP, EOFA_ERR_OOM):
            _check(rc)
        return rc, [s.as_dict() for s in stats]

    def gauge_shape(self):
        lx, ly, lz, lt = self.dims
        return (4, lt, lz, ly, lx, 3, 3)

    def eofa_cg_pairs(self, system, phi, npairs, first, stride, tol, max_iter, r_out, e_out, stream=None):
        """Training pairs (r_k, e_k) into r_out, e_out (uint8 tensors of npairs packed FP32 odd
        half-fields); returns (rc, recorded, iterations)."""
        rec, its = _I(0), _I(0)
        rc = lib().eofa_cg_pairs(self._h, make_systems([system]), _p(phi), npairs, first, stride, tol, max_iter,
                                 _p(r_out), _p(e_out), ctypes.byref(rec), ctypes.byref(its), _stream(stream))
        if rc in (EOFA_ERR_INVALID, EOFA_ERR_HIP, EOFA_ERR_OOM, EOFA_ERR_BREAKDOWN):
            _check(rc)
        return rc, rec.value, its.value


NET_TERMS = 20  # stencil terms per channel pair of a network layer


class Net:
    """An eofa_net: N = B^dag B with B a stack of gauge-covariant
    parallel-transport layers (device weights)."""

    def __init__(self, ctx, channels, seed=0, init_scale=1.0):
        self.channels = [int(c) for c in channels]
        ch = (_I * len(self.channels))(*self.channels)
        self._h = ctypes.c_void_p()
        _check(lib().eofa_net_create(ctx._h, len(self.channels) - 1, ch, seed, init_scale, ctypes.byref(self._h)))

    def close(self):
        if self._h:
            lib().eofa_net_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def num_weights(self):
        return int(lib().eofa_net_num_weights(self._h))

    def get_weights(self):
        """Complex weights as a list of [NET_TERMS, C_out, C_in] arrays (FP32 master values)."""
        n = self.num_weights()
        buf = (ctypes.c_double * (2 * n))()
        _check(lib().eofa_net_get_weights(self._h, buf))
        flat = np.frombuffer(buf, dtype=np.float64).copy()
        flat = flat[0::2] + 1j * flat[1::2]
        out, k = [], 0
        for ci, co in zip(self.channels[:-1], self.channels[1:]):
            out.append(flat[k:k + NET_TERMS * co * ci].reshape(NET_TERMS, co, ci))
            k += NET_TERMS * co * ci
        return out

    def set_weights(self, weights):
        flat = np.concatenate([np.asarray(w, dtype=np.complex128).ravel() for w in weights])
        assert flat.size == self.num_weights()
        buf = np.empty(2 * flat.size)
        buf[0::2], buf[1::2] = flat.real, flat.imag
        _check(lib().eofa_net_set_weights(self._h, buf.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))

    def apply(self, ctx, inp, out, stream=None):
        _check(lib().eofa_net_apply(ctx._h, self._h, _p(inp), _p(out), _stream(stream)))

    def loss_grad(self, ctx, r, e, npairs, system=None, stream=None):
        """(loss, [dL/dW* per layer]) over npairs packed FP32 pairs; with ``system``
        the scale-free residual loss 1 - |<A N(r), r>|^2/(|A N(r)|^2 |r|^2)
        summed over pairs (e unused), else the error loss |N(r) - e|^2/|e|^2."""
        n = self.num_weights()
        loss = ctypes.c_double()
        g = (ctypes.c_double * (2 * n))()
        _check(lib().eofa_net_loss_grad(ctx._h, self._h, _sys_or_null(system), _p(r), _p_or_null(e), npairs,
                                        ctypes.byref(loss), g, _stream(stream)))
        flat = np.frombuffer(g, dtype=np.float64).copy()
        flat = flat[0::2] + 1j * flat[1::2]
        out, k = [], 0
        for ci, co in zip(self.channels[:-1], self.channels[1:]):
            out.append(flat[k:k + NET_TERMS * co * ci].reshape(NET_TERMS, co, ci))
            k += NET_TERMS * co * ci
        return loss.value, out

    def train(self, ctx, r, e, npairs, epochs, batch, lr, system=None, stream=None):
        """Adam on the pairs (residual loss with ``system``); returns the mean loss
        per pair of every epoch."""
        hist = (ctypes.c_double * epochs)()
        _check(lib().eofa_net_train(ctx._h, self._h, _sys_or_null(system), _p(r), _p_or_null(e), npairs, epochs,
                                    batch, lr, hist, _stream(stream)))
        return list(hist)


def _p(t):
    return ctypes.c_void_p(t.data_ptr())


def _p_or_null(t):
    return None if t is None else _p(t)


def _sys_or_null(system):
    return None if system is None else make_systems([system])

"""ctypes binding of include/sg.h (same names, argument marshalling only).

Device arguments are torch CUDA (HIP) tensors of dtype float64 or raw integer
device addresses; `stream` is a torch.cuda.Stream, a raw hipStream_t integer,
or None for the current stream.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

HERE = os.path.dirname(os.path.abspath(__file__))

COV = {"exp_l1": 0, "sqexp": 1}
PC = {"none": 0, "mean": 1, "fs": 2, "learned": 3, "mg": 4, "mean_kii": 0x101, "fs_kii": 0x102,
      "learned_kii": 0x103, "mean_switch": 0x201, "fs_switch": 0x202}
GROUPING = {"klvar": 0, "klvar_meansep": 1, "permode": 2, "fg": 3, "all": 4}
EXPORT = {"coeff": 0, "kl": 1, "gq": 2, "stencil": 3, "groups": 4, "blocks": 5}
STATUS = {0: "converged", 1: "not_converged", 2: "breakdown"}
PC_INNER_SHIFT = 16


def pc_code(pc) -> int:
    """A preconditioner code from a name of PC, optionally ":k" for k inner
    iterations of the diagonal-block solves (e.g. "fs_kii:3"), or an int."""
    if isinstance(pc, str):
        name, _, k = pc.partition(":")
        return PC[name] | ((int(k) if k else 0) << PC_INNER_SHIFT)
    return int(pc)


class SGError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"sg error {code}: {msg}")
        self.code = code


class Problem(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("M", ctypes.c_int32), ("p", ctypes.c_int32),
                ("q", ctypes.c_int32), ("cov", ctypes.c_int32), ("mu", ctypes.c_double),
                ("sigma", ctypes.c_double), ("corr_len", ctypes.c_double),
                ("a_min", ctypes.c_double)]


class SolveOpts(ctypes.Structure):
    _fields_ = [("restart", ctypes.c_int32), ("max_it", ctypes.c_int32), ("pc", ctypes.c_int32),
                ("grouping", ctypes.c_int32), ("use_x0", ctypes.c_int32), ("tol", ctypes.c_double)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iterations", ctypes.c_int32),
                ("restarts", ctypes.c_int32), ("fallbacks", ctypes.c_int32),
                ("relres", ctypes.c_double), ("relres_est", ctypes.c_double)]


_lib = None


def library_path() -> str:
    return os.environ.get("SG_LIBRARY", os.path.join(HERE, "libsgfs.so"))


def load_library():
    """Loads libsgfs.so; raises if it is missing (there is no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    path = library_path()
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library not built: {path} is missing "
                           "(run python -m paper_1910_11505_amd.build)")
    lib = ctypes.CDLL(path)
    P, VP, SZ, I32, I64P = ctypes.POINTER, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int, ctypes.POINTER(ctypes.c_int64)
    HP = ctypes.c_void_p
    sig = {
        "sg_setup": (I32, [P(Problem), VP, P(HP)]),
        "sg_setup_q2": (I32, [P(Problem), VP, P(HP)]),
        "sg_sizes": (I32, [HP, I64P, I64P, I64P, I64P]),
        "sg_workspace_bytes": (SZ, [HP]),
        "sg_bind": (I32, [HP, VP, SZ, VP]),
        "sg_rhs": (I32, [HP, VP, VP]),
        "sg_apply": (I32, [HP, VP, VP, VP]),
        "sg_apply_noalloc": (I32, [HP, VP, VP, VP]),
        "sg_set_apply": (I32, [HP, I32, I32, VP]),
        "sg_apply_form": (I32, [HP, P(ctypes.c_int32), P(ctypes.c_int32)]),
        "sg_precond_apply": (I32, [HP, I32, I32, VP, VP, VP]),
        "sg_gmres_workspace_bytes": (SZ, [HP, P(SolveOpts)]),
        "sg_gmres_solve": (I32, [HP, P(SolveOpts), VP, VP, VP, SZ, VP, ctypes.c_int32,
                                 P(SolveInfo), VP]),
        "sg_export": (I32, [HP, I32, I32, VP, SZ]),
        "sg_destroy": (None, [HP]),
        "sg_last_error": (ctypes.c_char_p, []),
        "sg_cnn_create": (I32, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                ctypes.c_int32, P(HP)]),
        "sg_cnn_param_counts": (I32, [HP, I64P, I64P]),
        "sg_cnn_workspace_bytes": (SZ, [HP]),
        "sg_cnn_bind": (I32, [HP, VP, SZ, VP]),
        "sg_cnn_set_params": (I32, [HP, VP, VP, VP]),
        "sg_cnn_get_params": (I32, [HP, VP, VP]),
        "sg_cnn_get_adam": (I32, [HP, VP, VP, VP, VP]),
        "sg_cnn_set_adam": (I32, [HP, VP, VP, VP, VP, VP]),
        "sg_cnn_make_pair": (I32, [HP, VP, VP, VP, VP, VP, VP]),
        "sg_residual": (I32, [HP, VP, VP, VP, VP]),
        "sg_mg_workspace_bytes": (SZ, [HP, I32]),
        "sg_mg_bind": (I32, [HP, I32, VP, SZ, VP]),
        "sg_cnn_run": (I32, [HP, VP, VP, VP, VP, ctypes.c_int32, ctypes.c_int32, ctypes.c_float,
                             ctypes.c_int32, VP, ctypes.POINTER(ctypes.c_double), VP]),
        "sg_cnn_get_grads": (I32, [HP, VP, VP]),
        "sg_cnn_stage_work_doubles": (SZ, [HP]),
        "sg_cnn_stage_grad": (I32, [HP, HP, VP, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, VP,
                                    ctypes.POINTER(ctypes.c_double), VP]),
        "sg_cnn_backward": (I32, [HP, ctypes.c_int32, ctypes.c_int32, ctypes.c_float, ctypes.c_int32,
                                  VP]),
        "sg_cnn_apply": (I32, [HP, VP, ctypes.c_double, VP, VP]),
        "sg_cnn_destroy": (None, [HP]),
        "sg_cnn_last_error": (ctypes.c_char_p, []),
        "sg_attach_cnn": (I32, [HP, HP, ctypes.c_double]),
        "sg_batch_create": (I32, [ctypes.c_int32, P(Problem), VP, ctypes.c_int32, P(HP)]),
        "sg_batch_layout": (I32, [HP, I64P, VP]),
        "sg_batch_workspace_bytes": (SZ, [HP, ctypes.c_int32]),
        "sg_batch_bind": (I32, [HP, ctypes.c_int32, VP, SZ, VP]),
        "sg_batch_rhs": (I32, [HP, VP, VP]),
        "sg_batch_handle": (I32, [HP, ctypes.c_int32, P(HP)]),
        "sg_batch_solve": (I32, [HP, P(SolveOpts), VP, VP, P(SolveInfo), VP]),
        "sg_batch_destroy": (None, [HP]),
        "sg_autotune_apply": (I32, [P(Problem), ctypes.POINTER(ctypes.c_int32),
                                    ctypes.POINTER(ctypes.c_float)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _check(rc):
    if rc != 0:
        raise SGError(rc, load_library().sg_last_error().decode())


def _ptr(x):
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return x.data_ptr()


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def make_problem(n, M, p, q, cov="exp_l1", mu=0.0, sigma=0.5, corr_len=0.5, a_min=0.01):
    return Problem(n, M, p, q, COV[cov] if isinstance(cov, str) else int(cov), mu, sigma,
                   corr_len, a_min)


# ---- same names as the C ABI ------------------------------------------------
def sg_setup(prob: Problem, f_nodal=None):
    import numpy as np
    lib = load_library()
    h = ctypes.c_void_p()
    fp = None
    if f_nodal is not None:
        f_nodal = np.ascontiguousarray(f_nodal, dtype=np.float64)
        fp = f_nodal.ctypes.data
    _check(lib.sg_setup(ctypes.byref(prob), fp, ctypes.byref(h)))
    return h


def sg_setup_q2(prob: Problem, f_nodal=None):
    import numpy as np
    lib = load_library()
    h = ctypes.c_void_p()
    fp = None
    if f_nodal is not None:
        f_nodal = np.ascontiguousarray(f_nodal, dtype=np.float64)
        fp = f_nodal.ctypes.data
    _check(lib.sg_setup_q2(ctypes.byref(prob), fp, ctypes.byref(h)))
    return h


def sg_sizes(h):
    vals = [ctypes.c_int64() for _ in range(4)]
    _check(load_library().sg_sizes(h, *[ctypes.byref(v) for v in vals]))
    return tuple(v.value for v in vals)


def sg_workspace_bytes(h) -> int:
    return int(load_library().sg_workspace_bytes(h))


def sg_bind(h, ws, nbytes, stream=None):
    _check(load_library().sg_bind(h, _ptr(ws), nbytes, _stream(stream)))


def sg_rhs(h, F, stream=None):
    _check(load_library().sg_rhs(h, _ptr(F), _stream(stream)))


def sg_apply(h, U, W, stream=None):
    _check(load_library().sg_apply(h, _ptr(U), _ptr(W), _stream(stream)))


APPLY = {"auto": 0, "triple": 1, "factored": 2}


def sg_apply_form(h):
    """(form, points per sub-batch): form 2 register-resident, 1 factored LDS
    tiles, 0 triple products, 3 the biquadratic apply of a Q2 handle."""
    f, q = ctypes.c_int32(), ctypes.c_int32()
    _check(load_library().sg_apply_form(h, ctypes.byref(f), ctypes.byref(q)))
    return f.value, q.value


def sg_set_apply(h, kind="auto", points_per_batch=0, stream=None):
    kind = APPLY[kind] if isinstance(kind, str) else int(kind)
    _check(load_library().sg_set_apply(h, kind, int(points_per_batch), _stream(stream)))


def sg_precond_apply(h, pc, grouping, r, z, stream=None):
    pc = pc_code(pc)
    grouping = GROUPING[grouping] if isinstance(grouping, str) else int(grouping)
    _check(load_library().sg_precond_apply(h, pc, grouping, _ptr(r), _ptr(z), _stream(stream)))


def sg_gmres_workspace_bytes(h, opts: SolveOpts) -> int:
    return int(load_library().sg_gmres_workspace_bytes(h, ctypes.byref(opts)))


def sg_gmres_solve(h, opts: SolveOpts, F, u, ws, nbytes, hist=None, stream=None):
    info = SolveInfo()
    hp, hl = None, 0
    if hist is not None:
        hp, hl = hist.ctypes.data, len(hist)
    _check(load_library().sg_gmres_solve(h, ctypes.byref(opts), _ptr(F), _ptr(u), _ptr(ws), nbytes,
                                         hp, hl, ctypes.byref(info), _stream(stream)))
    return info


def sg_export(h, what, level, out):
    what = EXPORT[what] if isinstance(what, str) else int(what)
    _check(load_library().sg_export(h, what, level, out.ctypes.data, out.size))


def sg_destroy(h):
    load_library().sg_destroy(h)


def sg_last_error() -> str:
    return load_library().sg_last_error().decode()


def _ccheck(rc):
    if rc != 0:
        raise SGError(rc, load_library().sg_cnn_last_error().decode())


def sg_cnn_create(P, n, c0=32, c1=64, max_batch=16):
    h = ctypes.c_void_p()
    _ccheck(load_library().sg_cnn_create(P, n, c0, c1, max_batch, ctypes.byref(h)))
    return h


def sg_cnn_param_counts(c):
    a, b = ctypes.c_int64(), ctypes.c_int64()
    _ccheck(load_library().sg_cnn_param_counts(c, ctypes.byref(a), ctypes.byref(b)))
    return a.value, b.value


def sg_cnn_workspace_bytes(c) -> int:
    return int(load_library().sg_cnn_workspace_bytes(c))


def sg_cnn_bind(c, ws, nbytes, stream=None):
    _ccheck(load_library().sg_cnn_bind(c, _ptr(ws), nbytes, _stream(stream)))


def sg_cnn_set_params(c, w, b, stream=None):
    import numpy as np
    w = np.ascontiguousarray(w, dtype=np.float32)
    b = np.ascontiguousarray(b, dtype=np.float32)
    _ccheck(load_library().sg_cnn_set_params(c, w.ctypes.data, b.ctypes.data, _stream(stream)))


def sg_cnn_get_params(c, w, b):
    _ccheck(load_library().sg_cnn_get_params(c, w.ctypes.data, b.ctypes.data))


def sg_cnn_make_pair(c, r, ustar, u, R_out, T_out, stream=None):
    _ccheck(load_library().sg_cnn_make_pair(c, _ptr(r), _ptr(ustar), _ptr(u), _ptr(R_out),
                                            _ptr(T_out), _stream(stream)))


def sg_apply_noalloc(h, U, W, stream=None):
    _check(load_library().sg_apply_noalloc(h, _ptr(U), _ptr(W), _stream(stream)))


def sg_mg_workspace_bytes(h, grouping) -> int:
    grouping = GROUPING[grouping] if isinstance(grouping, str) else int(grouping)
    return int(load_library().sg_mg_workspace_bytes(h, grouping))


def sg_mg_bind(h, grouping, ws, nbytes, stream=None):
    grouping = GROUPING[grouping] if isinstance(grouping, str) else int(grouping)
    _check(load_library().sg_mg_bind(h, grouping, _ptr(ws), nbytes, _stream(stream)))


def sg_residual(h, F, u, r, stream=None):
    _check(load_library().sg_residual(h, _ptr(F), _ptr(u), _ptr(r), _stream(stream)))


def sg_cnn_run(c, R, T, sigma, idx, mode, lr=0.0, step=1, Y_out=None, want_loss=True, stream=None):
    import numpy as np
    idx = np.ascontiguousarray(idx, dtype=np.int32)
    loss = ctypes.c_double(0.0)
    _ccheck(load_library().sg_cnn_run(c, _ptr(R), _ptr(T), _ptr(sigma), idx.ctypes.data, len(idx),
                                      mode, lr, step, _ptr(Y_out),
                                      ctypes.byref(loss) if (want_loss and T is not None) else None,
                                      _stream(stream)))
    return loss.value


def sg_cnn_get_grads(c, dw, db):
    _ccheck(load_library().sg_cnn_get_grads(c, dw.ctypes.data, db.ctypes.data))


def sg_cnn_stage_work_doubles(h) -> int:
    return int(load_library().sg_cnn_stage_work_doubles(h))


def sg_cnn_stage_grad(h, c, R, pair, slot, batch, work, want_loss=False, stream=None):
    """The learned stage's objective for stored pair `pair` (batch slot `slot`
    of the last forward) with h's operator; returns it when want_loss."""
    loss = ctypes.c_double(0.0)
    _check(load_library().sg_cnn_stage_grad(h, c, _ptr(R), int(pair), int(slot), int(batch),
                                            _ptr(work), ctypes.byref(loss) if want_loss else None,
                                            _stream(stream)))
    return loss.value if want_loss else None


def sg_cnn_backward(c, batch, adam, lr=0.0, step=1, stream=None):
    _ccheck(load_library().sg_cnn_backward(c, int(batch), 1 if adam else 0, lr, int(step),
                                           _stream(stream)))


def sg_cnn_apply(c, v, sigma, out, stream=None):
    _ccheck(load_library().sg_cnn_apply(c, _ptr(v), sigma, _ptr(out), _stream(stream)))


def sg_cnn_destroy(c):
    load_library().sg_cnn_destroy(c)


def sg_cnn_last_error() -> str:
    return load_library().sg_cnn_last_error().decode()


def sg_attach_cnn(h, c, sigma):
    _check(load_library().sg_attach_cnn(h, c, sigma))


# ---- convenience owner of one bound instance ------------------------------
class SGInstance:
    """One problem bound to a device workspace owned by a torch uint8 tensor."""

    def __init__(self, n, M, p, q, cov="exp_l1", mu=0.0, sigma=0.5, corr_len=0.5, a_min=0.01,
                 f_nodal=None, device="cuda:0", stream=None, q2=False):
        """q2: biquadratic elements (sg_setup_q2), n elements per side."""
        import torch
        self.prob = make_problem(n, M, p, q, cov, mu, sigma, corr_len, a_min)
        self.q2 = q2
        self.h = (sg_setup_q2 if q2 else sg_setup)(self.prob, f_nodal)
        self.P, self.Nh, self.na, self.nnz = sg_sizes(self.h)
        self.device = torch.device(device)
        self.stream = stream
        nb = sg_workspace_bytes(self.h)
        self.ws = torch.empty(nb + 256, dtype=torch.uint8, device=self.device)
        off = (-self.ws.data_ptr()) % 256
        sg_bind(self.h, self.ws.data_ptr() + off, nb, stream)
        self._kws = None
        self._kws_key = None

    @property
    def nvec(self):
        return self.P * self.Nh

    def vec(self):
        import torch
        return torch.zeros(self.nvec, dtype=torch.float64, device=self.device)

    def rhs(self):
        F = self.vec()
        sg_rhs(self.h, F, self.stream)
        return F

    def apply(self, U, W=None):
        W = self.vec() if W is None else W
        sg_apply(self.h, U, W, self.stream)
        return W

    def apply_form(self):
        """(form, points per sub-batch) in use; see sg_apply_form."""
        return sg_apply_form(self.h)

    def set_apply(self, kind="auto", points_per_batch=0):
        """Apply form: "auto" (factored when q >= 2p), "triple" or "factored"."""
        sg_set_apply(self.h, kind, points_per_batch, self.stream)

    def precond(self, r, pc="mean", grouping="klvar", z=None):
        z = self.vec() if z is None else z
        sg_precond_apply(self.h, pc, grouping, r, z, self.stream)
        return z

    def solve(self, F=None, pc="fs", grouping="klvar", restart=50, max_it=5000, tol=1e-8,
              u=None, use_x0=False, hist_len=0):
        import numpy as np
        import torch
        F = self.rhs() if F is None else F
        u = self.vec() if u is None else u
        opts = SolveOpts(restart, max_it, pc_code(pc), GROUPING[grouping], 1 if use_x0 else 0, tol)
        nb = sg_gmres_workspace_bytes(self.h, opts)
        if self._kws is None or self._kws.numel() < nb + 256:
            self._kws = torch.empty(nb + 256, dtype=torch.uint8, device=self.device)
        off = (-self._kws.data_ptr()) % 256
        hist = np.zeros(hist_len) if hist_len else None
        info = sg_gmres_solve(self.h, opts, F, u, self._kws.data_ptr() + off, nb, hist, self.stream)
        return u, info, hist

    def export(self, what, level=0, count=None):
        import numpy as np
        if count is None:
            count = {"coeff": self.na * 4 * self.prob.n ** 2, "kl": self.prob.M,
                     "gq": self.prob.M * 4 * self.prob.n ** 2}.get(what)
        out = np.zeros(count)
        sg_export(self.h, what, level, out)
        return out

    def residual(self, F, u, r=None):
        r = self.vec() if r is None else r
        sg_residual(self.h, F, u, r, self.stream)
        return r

    def bind_mg(self, grouping="fg"):
        """Builds the full-system multigrid (pc="mg") for `grouping` in a device
        workspace owned by this instance."""
        import torch
        nb = sg_mg_workspace_bytes(self.h, grouping)
        if nb == 0:
            raise SGError(-1, "bad grouping for the full-system multigrid")
        self.mg_ws = torch.empty(nb + 256, dtype=torch.uint8, device=self.device)
        off = (-self.mg_ws.data_ptr()) % 256
        sg_mg_bind(self.h, grouping, self.mg_ws.data_ptr() + off, nb, self.stream)
        self.mg_grouping = grouping

    def attach(self, net, sigma):
        """Attaches a bound CNN (see CNN) for pc="learned" solves."""
        sg_attach_cnn(self.h, net.c if net is not None else None, sigma)

    def close(self):
        if self.h:
            sg_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class CNN:
    """Owner of one bound mode-channel network (device workspace in torch)."""

    def __init__(self, P, n, max_batch=16, device="cuda:0", stream=None, c0=32, c1=64):
        import torch
        self.P, self.n, self.c0, self.c1 = P, n, c0, c1
        self.c = sg_cnn_create(P, n, c0, c1, max_batch)
        self.nw, self.nb = sg_cnn_param_counts(self.c)
        self.device = torch.device(device)
        self.stream = stream
        nbytes = sg_cnn_workspace_bytes(self.c)
        self.ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        off = (-self.ws.data_ptr()) % 256
        sg_cnn_bind(self.c, self.ws.data_ptr() + off, nbytes, stream)

    def set_params(self, Ws, bs):
        import numpy as np
        sg_cnn_set_params(self.c, np.concatenate([w.reshape(-1) for w in Ws]),
                          np.concatenate([b.reshape(-1) for b in bs]), self.stream)

    def get_params(self):
        import numpy as np
        w = np.zeros(self.nw, dtype=np.float32)
        b = np.zeros(self.nb, dtype=np.float32)
        sg_cnn_get_params(self.c, w, b)
        return w, b

    def get_state(self):
        """Parameters and Adam moments (host copies): (w, b, wm, wv, bm, bv)."""
        import numpy as np
        w, b = self.get_params()
        wm, wv = np.zeros(self.nw, np.float32), np.zeros(self.nw, np.float32)
        bm, bv = np.zeros(self.nb, np.float32), np.zeros(self.nb, np.float32)
        _ccheck(load_library().sg_cnn_get_adam(self.c, wm.ctypes.data, wv.ctypes.data,
                                               bm.ctypes.data, bv.ctypes.data))
        return w, b, wm, wv, bm, bv

    def set_state(self, state):
        """Restores get_state()'s parameters and Adam moments."""
        import numpy as np
        w, b, wm, wv, bm, bv = (np.ascontiguousarray(x, dtype=np.float32) for x in state)
        sg_cnn_set_params(self.c, w, b, self.stream)
        _ccheck(load_library().sg_cnn_set_adam(self.c, wm.ctypes.data, wv.ctypes.data,
                                               bm.ctypes.data, bv.ctypes.data,
                                               _stream(self.stream)))

    def get_grads(self):
        import numpy as np
        w = np.zeros(self.nw, dtype=np.float32)
        b = np.zeros(self.nb, dtype=np.float32)
        sg_cnn_get_grads(self.c, w, b)
        return w, b

    def close(self):
        if self.c:
            sg_cnn_destroy(self.c)
            self.c = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def sg_autotune_apply(prob: Problem):
    kc = ctypes.c_int32(0)
    ms = ctypes.c_float(0.0)
    _check(load_library().sg_autotune_apply(ctypes.byref(prob), ctypes.byref(kc), ctypes.byref(ms)))
    return kc.value, ms.value


class Batch:
    """Many instances solved together by the batched persistent kernels."""

    def __init__(self, problems, f_nodal=None, restart=50, autotune=False, device="cuda:0",
                 stream=None):
        import numpy as np
        import torch
        self.count = len(problems)
        arr = (Problem * self.count)(*problems)
        self._f = None
        fp = None
        if f_nodal is not None:
            self._f = [None if f is None else np.ascontiguousarray(f, dtype=np.float64) for f in f_nodal]
            ptrs = (ctypes.c_void_p * self.count)(*[None if f is None else f.ctypes.data for f in self._f])
            fp = ctypes.cast(ptrs, ctypes.c_void_p)
            self._ptrs = ptrs
        self.b = ctypes.c_void_p()
        _check(load_library().sg_batch_create(self.count, arr, fp, 1 if autotune else 0,
                                              ctypes.byref(self.b)))
        self.offsets = np.zeros(self.count + 1, dtype=np.int64)
        self.form = np.zeros(self.count, dtype=np.int32)
        _check(load_library().sg_batch_layout(self.b, self.offsets.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                              self.form.ctypes.data))
        self.restart = restart
        self.device = torch.device(device)
        self.stream = stream
        nb = int(load_library().sg_batch_workspace_bytes(self.b, restart))
        self.ws = torch.empty(nb + 256, dtype=torch.uint8, device=self.device)
        off = (-self.ws.data_ptr()) % 256
        _check(load_library().sg_batch_bind(self.b, restart, self.ws.data_ptr() + off, nb,
                                            _stream(stream)))

    @property
    def total(self):
        return int(self.offsets[-1])

    def vec(self):
        import torch
        return torch.zeros(self.total, dtype=torch.float64, device=self.device)

    def rhs(self):
        F = self.vec()
        _check(load_library().sg_batch_rhs(self.b, F.data_ptr(), _stream(self.stream)))
        return F

    def handle(self, i):
        h = ctypes.c_void_p()
        _check(load_library().sg_batch_handle(self.b, i, ctypes.byref(h)))
        return h

    def solve(self, F, u=None, pc="fs", grouping="klvar", tol=1e-8, max_it=5000):
        u = self.vec() if u is None else u
        opts = SolveOpts(self.restart, max_it, pc_code(pc), GROUPING[grouping], 0, tol)
        infos = (SolveInfo * self.count)()
        _check(load_library().sg_batch_solve(self.b, ctypes.byref(opts), F.data_ptr(), u.data_ptr(),
                                             infos, _stream(self.stream)))
        return u, list(infos)

    def close(self):
        if self.b:
            load_library().sg_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

"""Thin ctypes binding of libtdo (C-ABI in include/tdo.h).

Argument marshalling only: torch tensors supply device memory and the current
HIP stream; every step of the computation runs in the library's kernels.
Loading fails loudly if the built library is missing; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtdo.so")

TDO_FP32, TDO_BF16 = 0, 1
PREC = {"fp32": TDO_FP32, "bf16": TDO_BF16}

# The entry points declared in include/tdo.h.
EXPORTS = ("tdo_ctx_create", "tdo_ctx_destroy", "tdo_num_params", "tdo_last_error", "tdo_profile",
           "tdo_profile_read", "tdo_connected", "tdo_local_lindbladian", "tdo_log_rho", "tdo_log_rho_vjp",
           "tdo_loss_grad", "tdo_loss_grad_batched", "tdo_sample", "tdo_sample_diag", "tdo_observables",
           "tdo_purity", "tdo_lr_schedule", "tdo_sgd_step", "tdo_adam_step", "tdo_log_rho_jacobian",
           "tdo_sr_solve", "tdo_log_rho_noalloc", "tdo_log_rho_jvp", "tdo_sr_solve_matfree", "tdo_autotune")


class ArchT(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int32) for k in ("d", "heads", "layers", "mlp", "c1", "act")]


class ModelT(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("n", ctypes.c_int32)] + [
        (k, ctypes.c_double) for k in ("V", "g", "Jx", "Jy", "Jz", "Bx", "By", "Bz", "gamma")] + [
        ("rows", ctypes.c_int32)]


class TdoError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"tdo error {code}: {msg}")
        self.code = code


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                               f"(paper_2502_20723_amd/csrc/build.sh)")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
        L.tdo_last_error.restype = ctypes.c_char_p
        L.tdo_num_params.restype = i64
        L.tdo_num_params.argtypes = [ctypes.POINTER(ArchT)]
        L.tdo_ctx_create.argtypes = [ctypes.POINTER(vp), i32, sz]
        L.tdo_ctx_destroy.argtypes = [vp]
        L.tdo_profile.argtypes = [vp, i32]
        L.tdo_profile_read.argtypes = [vp, ctypes.c_char_p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64)]
        L.tdo_connected.argtypes = [vp, ctypes.POINTER(ModelT), vp, i64, i32, vp, vp, vp, vp]
        L.tdo_local_lindbladian.argtypes = [vp, i64, vp, vp, vp, i32, vp, vp, vp]
        L.tdo_log_rho.argtypes = [vp, ctypes.POINTER(ArchT), vp, i32, vp, i64, i32, vp, vp]
        L.tdo_log_rho_noalloc.argtypes = [vp, ctypes.POINTER(ArchT), vp, i32, vp, i64, i32, vp, vp]
        L.tdo_log_rho_vjp.argtypes = [vp, ctypes.POINTER(ArchT), vp, i32, vp, i64, i32, vp, vp, vp]
        L.tdo_loss_grad.argtypes = [vp, ctypes.POINTER(ArchT), vp, ctypes.POINTER(ModelT), vp, i64, vp, i32, i32,
                                    vp, vp, vp, vp]
        L.tdo_loss_grad_batched.argtypes = [vp, ctypes.POINTER(ArchT), i32, ctypes.POINTER(ModelT), vp, vp, vp, vp, i32,
                                            i32, vp, vp, vp]
        L.tdo_sample.argtypes = [vp, ctypes.POINTER(ArchT), vp, i32, i64, vp, vp, ctypes.c_uint64,
                                 ctypes.POINTER(ctypes.c_uint64), i32, ctypes.c_float, i32, vp, vp]
        L.tdo_sample_diag.argtypes = [vp, ctypes.POINTER(ArchT), vp, i32, i64, vp, vp, ctypes.c_uint64,
                                      ctypes.POINTER(ctypes.c_uint64), i32, i32, vp, vp]
        L.tdo_observables.argtypes = [vp, ctypes.POINTER(ArchT), vp, i32, vp, i64, i32, vp, vp, vp, vp, vp]
        L.tdo_purity.argtypes = [vp, ctypes.POINTER(ArchT), vp, i32, vp, vp, i64, i32, vp, vp]
        dbl = ctypes.c_double
        L.tdo_lr_schedule.argtypes = [i64, dbl, i64, i64, dbl]
        L.tdo_sgd_step.argtypes = [i64, vp, vp, dbl, vp]
        L.tdo_adam_step.argtypes = [i64, vp, vp, vp, vp, i64, dbl, dbl, dbl, dbl, vp]
        L.tdo_log_rho_jacobian.argtypes = [vp, ctypes.POINTER(ArchT), vp, i32, vp, i64, i32, vp, vp]
        L.tdo_sr_solve.argtypes = [vp, vp, i64, i64, vp, vp, dbl, i32, vp, vp, vp]
        L.tdo_autotune.argtypes = [vp, ctypes.POINTER(ArchT), vp, ctypes.POINTER(ModelT), vp, i64, i32, i32, vp, vp,
                                   ctypes.POINTER(ctypes.c_int32), vp]
        L.tdo_log_rho_jvp.argtypes = [vp, ctypes.POINTER(ArchT), vp, i32, vp, i64, vp, vp, vp]
        L.tdo_sr_solve_matfree.argtypes = [vp, ctypes.POINTER(ArchT), vp, i32, vp, i64, vp, i32, vp, dbl, i32, vp, vp,
                                           vp]
        for name in EXPORTS:
            if name not in ("tdo_last_error", "tdo_num_params", "tdo_ctx_create", "tdo_ctx_destroy",
                            "tdo_lr_schedule"):
                getattr(L, name).restype = i32
        L.tdo_lr_schedule.restype = ctypes.c_double
        L.tdo_ctx_create.restype = i32
        L.tdo_ctx_destroy.restype = i32
        _lib = L
    return _lib


def _check(code):
    if code != 0:
        raise TdoError(code, lib().tdo_last_error().decode())


TDO_ENONFINITE = -5
TDO_ACT_RELU_FFN = 0


def arch_t(a: dict) -> ArchT:
    return ArchT(int(a["d"]), int(a["heads"]), int(a["layers"]), int(a["mlp"]), int(a.get("c1", 0) or 0),
                 int(a.get("act", TDO_ACT_RELU_FFN)))


def model_t(m: dict) -> ModelT:
    return ModelT(int(m["kind"]), int(m["n"]), *[float(m.get(k, 0.0) or 0.0) for k in
                                                 ("V", "g", "Jx", "Jy", "Jz", "Bx", "By", "Bz")],
                  float(m.get("gamma", 1.0)), int(m.get("rows", 1) or 1))


def lr_schedule(step: int, eta0: float, i_switch: int, i_decay: int, alpha: float) -> float:
    return float(lib().tdo_lr_schedule(step, eta0, i_switch, i_decay, alpha))


def sgd_step(params, grad, lr: float):
    """In place: params (device float32 [P]) -= lr grad (device float64 [P])."""
    P = params.shape[0]
    _dev(params, torch.float32, (P,), "params")
    _dev(grad, torch.float64, (P,), "grad")
    _check(lib().tdo_sgd_step(P, _ptr(params), _ptr(grad), lr, _stream()))


def adam_step(params, grad, m, v, t: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-8):
    """In place: one Adam step on params (device float32 [P]) with moments m, v
    (device float64 [P], zero before t = 1)."""
    P = params.shape[0]
    _dev(params, torch.float32, (P,), "params")
    for x, nm in ((grad, "grad"), (m, "m"), (v, "v")):
        _dev(x, torch.float64, (P,), nm)
    _check(lib().tdo_adam_step(P, _ptr(params), _ptr(grad), _ptr(m), _ptr(v), t, lr, beta1, beta2, eps,
                               _stream()))


def num_params(a: dict) -> int:
    p = lib().tdo_num_params(ctypes.byref(arch_t(a)))
    if p < 0:
        raise TdoError(-1, lib().tdo_last_error().decode())
    return int(p)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(t, dtype, shape=None, name="tensor"):
    if not (t.is_cuda and t.dtype == dtype and t.is_contiguous()):
        raise ValueError(f"{name} must be a contiguous CUDA {dtype} tensor")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return t


@dataclass
class Ctx:
    """A library context on one device with a workspace budget."""

    device: int = 0
    workspace_bytes: int = 0

    def __post_init__(self):
        h = ctypes.c_void_p()
        _check(lib().tdo_ctx_create(ctypes.byref(h), self.device, self.workspace_bytes))
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            _check(lib().tdo_ctx_destroy(self.h))
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------ profiling
    def profile(self, enable: bool):
        _check(lib().tdo_profile(self.h, int(bool(enable))))

    def profile_read(self, kernel: str):
        """(summed launch milliseconds, launch count) of a kernel group."""
        ms, k = ctypes.c_double(), ctypes.c_int64()
        _check(lib().tdo_profile_read(self.h, kernel.encode(), ctypes.byref(ms), ctypes.byref(k)))
        return float(ms.value), int(k.value)

    # ------------------------------------------------------------ entry points
    def connected(self, model: dict, cfg: torch.Tensor, kmax: int | None = None):
        n = int(model["n"])
        if kmax is None:
            fields = model.get("kind") == 1 and (model.get("Bx", 0) or model.get("By", 0))
            kmax = (5 if fields else 3) * n + 1
        B = cfg.shape[0]
        _dev(cfg, torch.uint64, (B, 2), "cfg")
        conn = torch.zeros((B, kmax, 2), dtype=torch.uint64, device=cfg.device)
        mel = torch.zeros((B, kmax, 2), dtype=torch.float32, device=cfg.device)
        ncon = torch.zeros((B,), dtype=torch.int32, device=cfg.device)
        _check(lib().tdo_connected(self.h, ctypes.byref(model_t(model)), _ptr(cfg), B, kmax, _ptr(conn), _ptr(mel),
                                   _ptr(ncon), _stream()))
        return conn, mel, ncon

    def local_lindbladian(self, lr_x, mel, ncon, lr_conn):
        B, kmax = mel.shape[0], mel.shape[1]
        _dev(lr_x, torch.float32, (B, 2), "log_rho_x")
        _dev(mel, torch.float32, (B, kmax, 2), "mel")
        _dev(ncon, torch.int32, (B,), "n_conn")
        _dev(lr_conn, torch.float32, (B, kmax, 2), "log_rho_conn")
        out = torch.empty((B, 2), dtype=torch.float32, device=mel.device)
        _check(lib().tdo_local_lindbladian(self.h, B, _ptr(lr_x), _ptr(mel), _ptr(ncon), kmax, _ptr(lr_conn),
                                           _ptr(out), _stream()))
        return out

    def log_rho(self, arch: dict, params, n: int, cfg, prec="fp32"):
        B = cfg.shape[0]
        _dev(params, torch.float32, (num_params(arch),), "params")
        _dev(cfg, torch.uint64, (B, 2), "cfg")
        out = torch.empty((B, 2), dtype=torch.float32, device=cfg.device)
        _check(lib().tdo_log_rho(self.h, ctypes.byref(arch_t(arch)), _ptr(params), n, _ptr(cfg), B, PREC[prec],
                                 _ptr(out), _stream()))
        return out

    def log_rho_noalloc(self, arch: dict, params, n: int, cfg, out, prec="fp32"):
        """log rho into the caller's out (device float32 [B, 2]) through the entry point that
        allocates no device memory."""
        B = cfg.shape[0]
        _dev(params, torch.float32, (num_params(arch),), "params")
        _dev(cfg, torch.uint64, (B, 2), "cfg")
        _dev(out, torch.float32, (B, 2), "out")
        _check(lib().tdo_log_rho_noalloc(self.h, ctypes.byref(arch_t(arch)), _ptr(params), n, _ptr(cfg), B,
                                         PREC[prec], _ptr(out), _stream()))
        return out

    def log_rho_vjp(self, arch: dict, params, n: int, cfg, seed, prec="fp32"):
        B = cfg.shape[0]
        _dev(params, torch.float32, (num_params(arch),), "params")
        _dev(cfg, torch.uint64, (B, 2), "cfg")
        _dev(seed, torch.float32, (B, 2), "seed")
        grad = torch.empty((num_params(arch),), dtype=torch.float64, device=cfg.device)
        _check(lib().tdo_log_rho_vjp(self.h, ctypes.byref(arch_t(arch)), _ptr(params), n, _ptr(cfg), B, PREC[prec],
                                     _ptr(seed), _ptr(grad), _stream()))
        return grad

    def loss_grad(self, arch: dict, params, model: dict, cfg, weights=None, prec="fp32", mode="B",
                  want_lloc=False):
        B = cfg.shape[0]
        P = num_params(arch)
        _dev(params, torch.float32, (P,), "params")
        _dev(cfg, torch.uint64, (B, 2), "cfg")
        if weights is not None:
            _dev(weights, torch.float64, (B,), "weights")
        loss = torch.empty((1,), dtype=torch.float64, device=cfg.device)
        grad = torch.empty((P,), dtype=torch.float64, device=cfg.device)
        lloc = torch.empty((B, 2), dtype=torch.float32, device=cfg.device) if want_lloc else None
        _check(lib().tdo_loss_grad(self.h, ctypes.byref(arch_t(arch)), _ptr(params), ctypes.byref(model_t(model)),
                                   _ptr(cfg), B, _ptr(weights), PREC[prec], {"B": 0, "A": 1}[mode], _ptr(loss),
                                   _ptr(grad), _ptr(lloc), _stream()))
        return loss, grad, lloc

    def autotune(self, arch: dict, params, model: dict, cfg, prec="bf16", mode="B"):
        """Tune the tile shapes of this problem's shape; returns (forward waves, forward
        workgroups per CU, feed-forward backward waves)."""
        B, P = cfg.shape[0], num_params(arch)
        _dev(params, torch.float32, (P,), "params")
        _dev(cfg, torch.uint64, (B, 2), "cfg")
        loss = torch.empty((1,), dtype=torch.float64, device=cfg.device)
        grad = torch.empty((P,), dtype=torch.float64, device=cfg.device)
        shapes = (ctypes.c_int32 * 3)()
        _check(lib().tdo_autotune(self.h, ctypes.byref(arch_t(arch)), _ptr(params), ctypes.byref(model_t(model)),
                                  _ptr(cfg), B, PREC[prec], {"B": 0, "A": 1}[mode], _ptr(loss), _ptr(grad), shapes,
                                  _stream()))
        return tuple(int(v) for v in shapes)

    def loss_grad_batched(self, arch: dict, params: list, models: list, cfgs: list, weights=None, prec="fp32",
                          mode="B", out=None):
        """Loss and gradient of several problems in one call.  out = (loss [n] float64
        tensor, list of n float64 [P] tensors) reuses the output buffers, which lets a
        repeated identical call replay its recorded graph."""
        k = len(params)
        if not (len(models) == len(cfgs) == k) or (weights is not None and len(weights) != k):
            raise ValueError("params, models, cfgs (and weights) must have one entry per problem")
        P = num_params(arch)
        for i in range(k):
            _dev(params[i], torch.float32, (P,), f"params[{i}]")
            _dev(cfgs[i], torch.uint64, (cfgs[i].shape[0], 2), f"cfg[{i}]")
            if weights is not None and weights[i] is not None:
                _dev(weights[i], torch.float64, (cfgs[i].shape[0],), f"weights[{i}]")
        dev = cfgs[0].device if k else torch.device("cuda")
        if out is None:
            loss = torch.empty((k,), dtype=torch.float64, device=dev)
            grads = [torch.empty((P,), dtype=torch.float64, device=dev) for _ in range(k)]
        else:
            loss, grads = out
            _dev(loss, torch.float64, (k,), "loss")
            for i in range(k):
                _dev(grads[i], torch.float64, (P,), f"grad[{i}]")
        vpa = ctypes.c_void_p * max(k, 1)
        mt = (ModelT * max(k, 1))(*[model_t(m) for m in models])
        bt = (ctypes.c_int64 * max(k, 1))(*[int(c.shape[0]) for c in cfgs])
        wt = None if weights is None else vpa(*[(w.data_ptr() if w is not None else None) for w in weights])
        _check(lib().tdo_loss_grad_batched(self.h, ctypes.byref(arch_t(arch)), k, mt, vpa(*[p.data_ptr() for p in params]),
                                           vpa(*[c.data_ptr() for c in cfgs]), bt, wt, PREC[prec], {"B": 0, "A": 1}[mode],
                                           _ptr(loss), vpa(*[g.data_ptr() for g in grads]), _stream()))
        return loss, grads

    def sample(self, arch: dict, params, n: int, state, state_lr, seed: int, counter: int, sweeps: int,
               p_pair=0.5, prec="fp32"):
        C = state.shape[0]
        _dev(params, torch.float32, (num_params(arch),), "params")
        _dev(state, torch.uint64, (C, 2), "state")
        _dev(state_lr, torch.float32, (C, 2), "state_log_rho")
        samples = torch.empty((sweeps, C, 2), dtype=torch.uint64, device=state.device)
        ctr = ctypes.c_uint64(counter)
        _check(lib().tdo_sample(self.h, ctypes.byref(arch_t(arch)), _ptr(params), n, C, _ptr(state), _ptr(state_lr),
                                seed, ctypes.byref(ctr), sweeps, p_pair, PREC[prec], _ptr(samples), _stream()))
        return samples, int(ctr.value)

    def jacobian(self, arch: dict, params, n: int, cfg, prec="fp32"):
        """O(x_b) = d log rho(x_b)/d theta as float64 [B, 2, P] (real, imaginary rows)."""
        B, P = cfg.shape[0], num_params(arch)
        _dev(params, torch.float32, (P,), "params")
        _dev(cfg, torch.uint64, (B, 2), "cfg")
        jac = torch.empty((B, 2, P), dtype=torch.float64, device=cfg.device)
        _check(lib().tdo_log_rho_jacobian(self.h, ctypes.byref(arch_t(arch)), _ptr(params), n, _ptr(cfg), B,
                                          PREC[prec], _ptr(jac), _stream()))
        return jac

    def sr_solve(self, jac, grad, lam: float, iters: int, weights=None):
        """x = (S + lam I)^-1 grad by conjugate gradients; jac ([B, 2, P] float64) is
        centred and scaled in place.  Returns (x, info [rel. residual, |g|])."""
        B, _, P = jac.shape
        _dev(jac, torch.float64, (B, 2, P), "jac")
        _dev(grad, torch.float64, (P,), "grad")
        if weights is not None:
            _dev(weights, torch.float64, (B,), "weights")
        x = torch.empty((P,), dtype=torch.float64, device=jac.device)
        info = torch.empty((2,), dtype=torch.float64, device=jac.device)
        _check(lib().tdo_sr_solve(self.h, _ptr(jac), B, P, _ptr(weights), _ptr(grad), lam, iters, _ptr(x),
                                  _ptr(info), _stream()))
        return x, info

    def log_rho_jvp(self, arch: dict, params, n: int, cfg, tangent):
        """d log rho(x_b) along tangent (device float64 [P]) as float32 [B, 2] (re, im)."""
        B, P = cfg.shape[0], num_params(arch)
        _dev(params, torch.float32, (P,), "params")
        _dev(cfg, torch.uint64, (B, 2), "cfg")
        _dev(tangent, torch.float64, (P,), "tangent")
        out = torch.empty((B, 2), dtype=torch.float32, device=cfg.device)
        _check(lib().tdo_log_rho_jvp(self.h, ctypes.byref(arch_t(arch)), _ptr(params), n, _ptr(cfg), B, _ptr(tangent),
                                     _ptr(out), _stream()))
        return out

    def sr_solve_matfree(self, arch: dict, params, n: int, cfg, grad, lam: float, iters: int, weights=None,
                         prec="fp32"):
        """x = (S + lam I)^-1 grad with S applied as J^T (J p) (no Jacobian stored).
        Returns (x, info [rel. residual, |g|])."""
        B, P = cfg.shape[0], num_params(arch)
        _dev(params, torch.float32, (P,), "params")
        _dev(cfg, torch.uint64, (B, 2), "cfg")
        _dev(grad, torch.float64, (P,), "grad")
        if weights is not None:
            _dev(weights, torch.float64, (B,), "weights")
        x = torch.empty((P,), dtype=torch.float64, device=cfg.device)
        info = torch.empty((2,), dtype=torch.float64, device=cfg.device)
        _check(lib().tdo_sr_solve_matfree(self.h, ctypes.byref(arch_t(arch)), _ptr(params), n, _ptr(cfg), B,
                                          _ptr(weights), PREC[prec], _ptr(grad), lam, iters, _ptr(x), _ptr(info),
                                          _stream()))
        return x, info

    def sample_diag(self, arch: dict, params, n: int, state, state_lr, seed: int, counter: int, sweeps: int,
                    prec="fp32"):
        C = state.shape[0]
        _dev(params, torch.float32, (num_params(arch),), "params")
        _dev(state, torch.uint64, (C,), "state")
        _dev(state_lr, torch.float32, (C, 2), "state_log_rho")
        samples = torch.empty((sweeps, C), dtype=torch.uint64, device=state.device)
        ctr = ctypes.c_uint64(counter)
        _check(lib().tdo_sample_diag(self.h, ctypes.byref(arch_t(arch)), _ptr(params), n, C, _ptr(state),
                                     _ptr(state_lr), seed, ctypes.byref(ctr), sweeps, PREC[prec], _ptr(samples),
                                     _stream()))
        return samples, int(ctr.value)

    def observables(self, arch: dict, params, n: int, alpha, prec="fp32", want_mean=True, want_sites=False):
        """(log rho(alpha, alpha) [B, 2], local estimators [B, 3, 2] (x, y, z site averages),
        sign-weighted means [7] float64 or None); with want_sites, also the per-site
        estimators [B, n, 3, 2] as a fourth element."""
        B = alpha.shape[0]
        _dev(params, torch.float32, (num_params(arch),), "params")
        _dev(alpha, torch.uint64, (B,), "alpha")
        lrd = torch.empty((B, 2), dtype=torch.float32, device=alpha.device)
        local = torch.empty((B, 3, 2), dtype=torch.float32, device=alpha.device)
        mean = torch.empty((7,), dtype=torch.float64, device=alpha.device) if want_mean else None
        site = torch.empty((B, n, 3, 2), dtype=torch.float32, device=alpha.device) if want_sites else None
        _check(lib().tdo_observables(self.h, ctypes.byref(arch_t(arch)), _ptr(params), n, _ptr(alpha), B,
                                     PREC[prec], _ptr(lrd), _ptr(local), _ptr(site), _ptr(mean), _stream()))
        return (lrd, local, mean, site) if want_sites else (lrd, local, mean)

    def purity(self, arch: dict, params, n: int, alpha, beta, prec="fp32"):
        """[purity estimate, mean sign] (float64, device) from pairs (alpha_p, beta_p)."""
        P = alpha.shape[0]
        _dev(params, torch.float32, (num_params(arch),), "params")
        _dev(alpha, torch.uint64, (P,), "alpha")
        _dev(beta, torch.uint64, (P,), "beta")
        out = torch.empty((2,), dtype=torch.float64, device=alpha.device)
        _check(lib().tdo_purity(self.h, ctypes.byref(arch_t(arch)), _ptr(params), n, _ptr(alpha), _ptr(beta), P,
                                PREC[prec], _ptr(out), _stream()))
        return out


_default_ctx = None


def default_ctx() -> Ctx:
    global _default_ctx
    if _default_ctx is None:
        _default_ctx = Ctx(torch.cuda.current_device())
    return _default_ctx


class LogRho(torch.autograd.Function):
    """log rho (complex as [B, 2] float) with the library's backward as VJP."""

    @staticmethod
    def forward(ctx, params, arch, n, cfg, prec):
        ctx.save_for_backward(params, cfg)
        ctx.arch, ctx.n, ctx.prec = arch, n, prec
        return default_ctx().log_rho(arch, params, n, cfg, prec)

    @staticmethod
    def backward(ctx, g):
        params, cfg = ctx.saved_tensors
        grad = default_ctx().log_rho_vjp(ctx.arch, params, ctx.n, cfg, g.contiguous().float(), ctx.prec)
        return grad.to(params.dtype), None, None, None, None


class LossGrad(torch.autograd.Function):
    """Cost of the samples; its backward returns the library's gradient
    estimator (mode B by default) times the upstream scalar."""

    @staticmethod
    def forward(ctx, params, arch, model, cfg, weights, prec, mode):
        loss, grad, _ = default_ctx().loss_grad(arch, params, model, cfg, weights, prec, mode)
        ctx.save_for_backward(grad)
        return loss[0]

    @staticmethod
    def backward(ctx, g):
        (grad,) = ctx.saved_tensors
        return (g.double() * grad).to(torch.float32), None, None, None, None, None, None

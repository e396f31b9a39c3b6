"""Thin ctypes binding of the C ABI in include/ga.h (same names, argument
marshalling only).  Vectors are torch tensors on the GPU (FP64, contiguous);
the library does all the compute.  Loading fails loudly if libga.so has not
been built: there is no fallback path."""
import ctypes
import os

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libga.so")

GA_OK, GA_EINVAL, GA_ENOMEM, GA_EDEVICE, GA_EGEOMETRY, GA_ENOCONV, GA_EUNSTABLE = 0, -1, -2, -3, -4, -5, -6
GA_GUESS_ZERO, GA_GUESS_PREV, GA_GUESS_EXTRAP, GA_GUESS_LEARNED = 0, 1, 2, 3
GA_GNET_NPARAM = 32033
GA_FP64, GA_FP32, GA_BF16 = 0, 1, 2
GA_PINV_AUTO, GA_PINV_DENSE, GA_PINV_MFMA = 0, 1, 2
GA_CG_HOST, GA_CG_DEVICE, GA_CG_FUSED = 0, 1, 2

EXPORTS = ["ga_setup_patch", "ga_setup_patch_ex", "ga_destroy_patch", "ga_patch_info", "ga_diag_M", "ga_apply_MK",
           "ga_apply_Pinv", "ga_apply_Pinv_noalloc", "ga_mass_solve", "ga_lambda_max", "ga_stability_limit",
           "ga_integrator_create", "ga_integrator_destroy", "ga_init_state", "ga_step",
           "ga_profile", "ga_profile_query", "ga_solve_stats", "ga_last_error", "ga_stage_solution", "ga_patch_set_pinv",
           "ga_integrator_set_damping", "ga_stage_times", "ga_init_state_forced", "ga_step_forced",
           "ga_gnet_create", "ga_gnet_destroy", "ga_gnet_set_params", "ga_gnet_get_params",
           "ga_gnet_set_train_prec",
           "ga_gnet_make_batch", "ga_gnet_forward", "ga_gnet_loss_grad", "ga_gnet_adam", "ga_gnet_infer",
           "ga_integrator_set_net", "ga_integrator_history", "ga_integrator_set_history", "ga_batch_create", "ga_batch_destroy", "ga_batch_info",
           "ga_batch_tune", "ga_batch_set_precision", "ga_batch_set_tau", "ga_patch_set_cg", "ga_cg_stats", "ga_patch_tune", "ga_patch_tuned_layers", "ga_patch_set_layers", "ga_patch_set_deterministic",
           "ga_stability_limit2", "ga_integrator_set_rho", "ga_wave1d_create", "ga_wave1d_destroy",
           "ga_wave1d_info", "ga_wave1d_load_sine", "ga_wave1d_apply", "ga_wave1d_init_state",
           "ga_wave1d_step", "ga_batch_init_state", "ga_batch_step", "ga_mp_create", "ga_mp_destroy",
           "ga_mp_info", "ga_mp_apply", "ga_mp_mass_solve", "ga_mp_init_state", "ga_mp_step"]


class GAError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"ga error {code}: {msg}")
        self.code = code


_lib = None


def load_library(path=LIB_PATH):
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with __graft_entry__.build() "
                           "(the HIP library is the only compute path)")
    lib = ctypes.CDLL(path)
    vp, i, d, dp = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_void_p
    lib.ga_setup_patch.argtypes = [i, ctypes.POINTER(i), i, ctypes.POINTER(d), vp, ctypes.POINTER(vp)]
    lib.ga_setup_patch_ex.argtypes = [i, ctypes.POINTER(i), i, ctypes.POINTER(d), ctypes.c_uint, vp,
                                      ctypes.POINTER(vp)]
    lib.ga_destroy_patch.argtypes = [vp]
    lib.ga_patch_info.argtypes = [vp, ctypes.POINTER(ctypes.c_longlong), ctypes.POINTER(ctypes.c_longlong),
                                  ctypes.POINTER(i)]
    lib.ga_diag_M.argtypes = [vp, dp, vp]
    lib.ga_apply_MK.argtypes = [vp, ctypes.c_char, i, i, d, dp, dp, vp]
    lib.ga_apply_Pinv.argtypes = [vp, i, i, dp, dp, vp]
    lib.ga_apply_Pinv_noalloc.argtypes = [vp, i, dp, dp, vp]
    lib.ga_mass_solve.argtypes = [vp, i, dp, dp, d, i, i, ctypes.POINTER(i), ctypes.POINTER(d), vp]
    lib.ga_lambda_max.argtypes = [vp, i, ctypes.POINTER(d), vp]
    lib.ga_stability_limit.argtypes = [d]
    lib.ga_stability_limit.restype = d
    lib.ga_integrator_create.argtypes = [vp, i, d, d, d, i, i, i, ctypes.POINTER(vp)]
    lib.ga_integrator_destroy.argtypes = [vp]
    lib.ga_init_state.argtypes = [vp, dp, dp, ctypes.POINTER(vp), vp]
    lib.ga_step.argtypes = [vp, ctypes.POINTER(vp), i, ctypes.POINTER(i), vp]
    lib.ga_solve_stats.argtypes = [vp, ctypes.POINTER(ctypes.c_longlong), ctypes.POINTER(ctypes.c_longlong),
                                   ctypes.POINTER(ctypes.c_longlong), ctypes.POINTER(d), i]
    lib.ga_profile.argtypes = [i]
    lib.ga_profile_query.argtypes = [i, ctypes.POINTER(d), ctypes.POINTER(ctypes.c_longlong)]
    lib.ga_last_error.argtypes = []
    lib.ga_last_error.restype = ctypes.c_char_p
    ip, fp = ctypes.POINTER(i), ctypes.POINTER(ctypes.c_float)
    lib.ga_stage_solution.argtypes = [vp, i, i, dp, vp]
    lib.ga_patch_set_pinv.argtypes = [vp, i]
    lib.ga_patch_set_cg.argtypes = [vp, i]
    lib.ga_patch_tune.argtypes = [vp, i, i, ctypes.POINTER(d), vp]
    lib.ga_patch_tuned_layers.argtypes = [vp, ctypes.POINTER(i), ctypes.POINTER(i)]
    lib.ga_patch_set_layers.argtypes = [vp, i, i]
    lib.ga_patch_set_deterministic.argtypes = [vp, i]
    lib.ga_cg_stats.argtypes = [vp, ctypes.POINTER(ctypes.c_longlong), ctypes.POINTER(ctypes.c_longlong)]
    lib.ga_integrator_set_damping.argtypes = [vp, d, d]
    lib.ga_stage_times.argtypes = [vp, d, ctypes.POINTER(d)]
    lib.ga_init_state_forced.argtypes = [vp, dp, dp, ctypes.POINTER(vp), ctypes.POINTER(vp), vp]
    lib.ga_step_forced.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(i), vp]
    lib.ga_gnet_create.argtypes = [fp, ctypes.POINTER(vp)]
    lib.ga_gnet_destroy.argtypes = [vp]
    lib.ga_gnet_set_params.argtypes = [vp, fp]
    lib.ga_gnet_get_params.argtypes = [vp, fp]
    lib.ga_gnet_set_train_prec.argtypes = [vp, i]
    lib.ga_gnet_make_batch.argtypes = [vp, vp, ctypes.POINTER(vp), dp, i, i, ip, dp, dp, vp]
    lib.ga_gnet_forward.argtypes = [vp, i, i, ip, ip, dp, dp, vp]
    lib.ga_gnet_loss_grad.argtypes = [vp, i, i, ip, ip, dp, dp, dp, ctypes.POINTER(d), vp]
    lib.ga_gnet_adam.argtypes = [vp, dp, ctypes.c_float, vp]
    lib.ga_gnet_infer.argtypes = [vp, vp, ctypes.POINTER(vp), dp, vp]
    lib.ga_integrator_set_net.argtypes = [vp, i, vp]
    lib.ga_integrator_history.argtypes = [vp, ctypes.POINTER(i)]
    lib.ga_integrator_set_history.argtypes = [vp, i, ctypes.POINTER(vp), vp]
    lp = ctypes.POINTER(ctypes.c_longlong)
    lib.ga_batch_create.argtypes = [i, ctypes.POINTER(vp), i, d, d, d, i, ctypes.POINTER(vp)]
    lib.ga_batch_destroy.argtypes = [vp]
    lib.ga_batch_info.argtypes = [vp, lp, lp, lp]
    lib.ga_batch_tune.argtypes = [vp, i, ctypes.POINTER(d), vp]
    lib.ga_batch_set_precision.argtypes = [vp, i, vp]
    lib.ga_batch_set_tau.argtypes = [vp, ctypes.POINTER(d)]
    lib.ga_batch_init_state.argtypes = [vp, dp, dp, ctypes.POINTER(vp), vp]
    lib.ga_batch_step.argtypes = [vp, ctypes.POINTER(vp), i, i, ctypes.POINTER(i), vp]
    lib.ga_mp_create.argtypes = [ctypes.POINTER(i), i, i, ctypes.POINTER(vp), i, d, d, d, i, vp,
                                 ctypes.POINTER(vp)]
    lib.ga_mp_destroy.argtypes = [vp]
    lib.ga_mp_info.argtypes = [vp, lp, ctypes.POINTER(i), lp]
    lib.ga_mp_apply.argtypes = [vp, ctypes.c_char, i, dp, dp, vp]
    lib.ga_mp_mass_solve.argtypes = [vp, i, dp, dp, ctypes.POINTER(i), vp]
    lib.ga_mp_init_state.argtypes = [vp, dp, dp, ctypes.POINTER(vp), vp]
    lib.ga_mp_step.argtypes = [vp, ctypes.POINTER(vp), i, ctypes.POINTER(i), vp]
    lib.ga_stability_limit2.argtypes = [d, d]
    lib.ga_stability_limit2.restype = d
    lib.ga_integrator_set_rho.argtypes = [vp, d, d]
    lib.ga_wave1d_create.argtypes = [i, i, i, ctypes.POINTER(d), i, d, d, d, ctypes.POINTER(vp)]
    lib.ga_wave1d_destroy.argtypes = [vp]
    lib.ga_wave1d_info.argtypes = [vp, ctypes.POINTER(i)]
    lib.ga_wave1d_load_sine.argtypes = [vp, ctypes.POINTER(d), dp, vp]
    lib.ga_wave1d_apply.argtypes = [vp, ctypes.c_char, dp, dp, vp]
    lib.ga_wave1d_init_state.argtypes = [vp, dp, dp, ctypes.POINTER(vp), vp]
    lib.ga_wave1d_step.argtypes = [vp, ctypes.POINTER(vp), i, vp]
    for name in EXPORTS:
        if name not in ("ga_stability_limit", "ga_stability_limit2", "ga_last_error"):
            getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _check(rc):
    if rc != GA_OK:
        raise GAError(rc, _lib.ga_last_error().decode())
    return rc


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t, n=None):
    if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise ValueError("vectors must be contiguous float64 CUDA tensors")
    if n is not None and t.numel() < n:
        raise ValueError(f"vector has {t.numel()} entries, needs {n}")
    return ctypes.c_void_p(t.data_ptr())


class Patch:
    """One spline patch (ga_setup_patch)."""

    def __init__(self, dim, n_el, p, ctrl, dirichlet_faces=None):
        lib = load_library()
        n_el = [int(v) for v in (n_el if np.ndim(n_el) else [n_el] * dim)]
        ctrl = np.ascontiguousarray(ctrl, dtype=np.float64)
        arr = (ctypes.c_int * len(n_el))(*n_el)
        h = ctypes.c_void_p()
        cp = ctrl.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        if dirichlet_faces is None:
            _check(lib.ga_setup_patch(dim, arr, p, cp, _stream(), ctypes.byref(h)))
        else:
            _check(lib.ga_setup_patch_ex(dim, arr, p, cp, ctypes.c_uint(int(dirichlet_faces)), _stream(),
                                         ctypes.byref(h)))
        self.h = h
        nf, nq = ctypes.c_longlong(), ctypes.c_longlong()
        mf = (ctypes.c_int * 3)()
        _check(lib.ga_patch_info(h, ctypes.byref(nf), ctypes.byref(nq), mf))
        self.dim, self.p, self.n_el = dim, p, n_el
        self.n_free, self.n_quad, self.mf = nf.value, nq.value, tuple(mf)

    def close(self):
        if getattr(self, "h", None):
            _lib.ga_destroy_patch(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def ga_setup_patch(dim, n_el, p, ctrl):
    return Patch(dim, n_el, p, ctrl)


def ga_setup_patch_ex(dim, n_el, p, ctrl, dirichlet_faces):
    return Patch(dim, n_el, p, ctrl, dirichlet_faces)


def ga_patch_set_pinv(patch, mode):
    _check(_lib.ga_patch_set_pinv(patch.h, int(mode)))


def ga_patch_tune(patch, nrhs=2, reps=3):
    """Autotune the element layers per workgroup of the patch's mass and stiffness
    launches; returns the summed time of one tuned launch of each (ms)."""
    ms = ctypes.c_double()
    _check(_lib.ga_patch_tune(patch.h, int(nrhs), int(reps), ctypes.byref(ms), _stream()))
    return ms.value


def ga_patch_tuned_layers(patch):
    a, b = ctypes.c_int(), ctypes.c_int()
    _check(_lib.ga_patch_tuned_layers(patch.h, ctypes.byref(a), ctypes.byref(b)))
    return a.value, b.value


def ga_patch_set_layers(patch, ze_mass, ze_stiff):
    """Element layers per workgroup of the FP64 mass and stiffness launches (0: automatic)."""
    _check(_lib.ga_patch_set_layers(patch.h, int(ze_mass), int(ze_stiff)))


def ga_patch_set_deterministic(patch, on=True):
    """Fixed-order (colour-class) operator launches: bitwise reproducible results."""
    _check(_lib.ga_patch_set_deterministic(patch.h, int(bool(on))))


def ga_patch_set_cg(patch, mode):
    """GA_CG_HOST or GA_CG_DEVICE control of the patch's FP64 PCG solves."""
    _check(_lib.ga_patch_set_cg(patch.h, int(mode)))


def ga_cg_stats(patch):
    """(iterations enqueued ahead of a convergence read, host reads of the flags)."""
    a, b = ctypes.c_longlong(), ctypes.c_longlong()
    _check(_lib.ga_cg_stats(patch.h, ctypes.byref(a), ctypes.byref(b)))
    return a.value, b.value


def ga_diag_M(patch, d):
    _check(_lib.ga_diag_M(patch.h, _ptr(d, patch.n_free), _stream()))


def ga_apply_MK(patch, which, x, y, nrhs=1, alpha=1.0, prec=GA_FP64):
    n = nrhs * patch.n_free
    _check(_lib.ga_apply_MK(patch.h, which.encode(), nrhs, int(prec), float(alpha), _ptr(x, n), _ptr(y, n),
                            _stream()))


def ga_apply_Pinv(patch, r, z, nrhs=1, prec=GA_FP64):
    n = nrhs * patch.n_free
    _check(_lib.ga_apply_Pinv(patch.h, nrhs, int(prec), _ptr(r, n), _ptr(z, n), _stream()))


def ga_apply_Pinv_noalloc(patch, r, z, nrhs=1):
    """FP64 P^{-1} with the library's fixed device scratch (no allocation)."""
    n = nrhs * patch.n_free
    _check(_lib.ga_apply_Pinv_noalloc(patch.h, nrhs, _ptr(r, n), _ptr(z, n), _stream()))


GA_NOALLOC_MAX_ENTRIES = 4718592


def ga_mass_solve(patch, b, x, nrhs=1, rtol=1e-12, maxit=500, raise_on_noconv=True, prec=GA_FP64):
    """Returns (iterations[nrhs], relres[nrhs], status)."""
    n = nrhs * patch.n_free
    its = (ctypes.c_int * nrhs)()
    rel = (ctypes.c_double * nrhs)()
    rc = _lib.ga_mass_solve(patch.h, nrhs, _ptr(b, n), _ptr(x, n), float(rtol), int(maxit), int(prec),
                            its, rel, _stream())
    if rc != GA_ENOCONV or raise_on_noconv:
        _check(rc)
    return list(its), list(rel), rc


def ga_lambda_max(patch, iters=30):
    out = ctypes.c_double()
    _check(_lib.ga_lambda_max(patch.h, int(iters), ctypes.byref(out), _stream()))
    return out.value


def ga_stability_limit(rho):
    return load_library().ga_stability_limit(float(rho))


def ga_stability_limit2(rho_b, rho_s):
    return load_library().ga_stability_limit2(float(rho_b), float(rho_s))


def ga_integrator_set_rho(integ, rho_b, rho_s):
    """Two-parameter family 0 <= rho_s <= rho_b < 1 for an existing integrator."""
    _check(_lib.ga_integrator_set_rho(integ.h, float(rho_b), float(rho_s)))


class Integrator:
    def __init__(self, patch, k, rho, tau, rtol=1e-10, maxit=200, guess=GA_GUESS_ZERO, prec=GA_FP64):
        h = ctypes.c_void_p()
        _check(_lib.ga_integrator_create(patch.h, k, float(rho), float(tau), float(rtol), int(maxit),
                                         int(prec), int(guess), ctypes.byref(h)))
        self.h, self.patch, self.k = h, patch, k

    def close(self):
        if getattr(self, "h", None):
            _lib.ga_integrator_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def ga_integrator_create(patch, k, rho, tau, rtol=1e-10, maxit=200, guess=GA_GUESS_ZERO, prec=GA_FP64):
    return Integrator(patch, k, rho, tau, rtol, maxit, guess, prec)


def _state_array(integ, state):
    ns = 3 * integ.k
    if len(state) != ns:
        raise ValueError(f"need {ns} state vectors")
    return (ctypes.c_void_p * ns)(*[_ptr(s, integ.patch.n_free).value for s in state])


def ga_init_state(integ, U0, V0, state):
    n = integ.patch.n_free
    _check(_lib.ga_init_state(integ.h, _ptr(U0, n), _ptr(V0, n), _state_array(integ, state), _stream()))


def ga_integrator_set_damping(integ, cM, cK):
    _check(_lib.ga_integrator_set_damping(integ.h, float(cM), float(cK)))


def ga_stage_times(integ, t):
    out = (ctypes.c_double * integ.k)()
    _check(_lib.ga_stage_times(integ.h, float(t), out))
    return list(out)


def _vec_array(integ, vecs, count):
    if len(vecs) != count:
        raise ValueError(f"need {count} vectors")
    return (ctypes.c_void_p * count)(*[_ptr(v, integ.patch.n_free).value for v in vecs])


def ga_init_state_forced(integ, U0, V0, F0, state):
    """F0: list of 3k-2 device vectors F^{(a)}(0), a = 0..3k-3, or None."""
    n = integ.patch.n_free
    f = None if F0 is None else _vec_array(integ, F0, 3 * integ.k - 2)
    _check(_lib.ga_init_state_forced(integ.h, _ptr(U0, n), _ptr(V0, n), f, _state_array(integ, state),
                                     _stream()))


def ga_step_forced(integ, state, forcing):
    """One step; forcing: k device vectors F^{(a_j)} at the stage times."""
    its = (ctypes.c_int * integ.k)()
    _check(_lib.ga_step_forced(integ.h, _state_array(integ, state), _vec_array(integ, forcing, integ.k), its,
                               _stream()))
    return list(its)


def ga_step(integ, state, nsteps=1, record_iters=True):
    """Advance; returns an int array [nsteps, k] of PCG iterations (or None)."""
    its = (ctypes.c_int * (nsteps * integ.k))() if record_iters else None
    _check(_lib.ga_step(integ.h, _state_array(integ, state), int(nsteps), its, _stream()))
    return np.array(its, dtype=np.int64).reshape(nsteps, integ.k) if record_iters else None


PROF_MASS, PROF_STIFF, PROF_PINV, PROF_GUESS = 0, 1, 2, 3
GA_PROF_ALL = 15


def ga_profile(enable, kinds=None):
    """Time launches of `kinds` (PROF_* values; all four when None) while enabled."""
    mask = 0
    if enable:
        mask = GA_PROF_ALL if kinds is None else sum(1 << int(kd) for kd in set(kinds))
    _check(load_library().ga_profile(mask))


def ga_profile_query(kind):
    """(total_ms, launches) of one launch kind since the last ga_profile()."""
    ms, cnt = ctypes.c_double(), ctypes.c_longlong()
    _check(_lib.ga_profile_query(int(kind), ctypes.byref(ms), ctypes.byref(cnt)))
    return ms.value, cnt.value


def ga_solve_stats(patch, reset=True):
    """dict(solves, guessed, fallbacks, mean_guess_relres) since the last reset."""
    a, b, c = ctypes.c_longlong(), ctypes.c_longlong(), ctypes.c_longlong()
    m = ctypes.c_double()
    _check(_lib.ga_solve_stats(patch.h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c), ctypes.byref(m),
                               1 if reset else 0))
    return {"solves": a.value, "guessed": b.value, "fallbacks": c.value, "mean_guess_relres": m.value}


def ga_stage_solution(integ, stage, age, out):
    _check(_lib.ga_stage_solution(integ.h, int(stage), int(age), _ptr(out, integ.patch.n_free), _stream()))


# ---- learned initial guess ----

def _fptr(t, n=None):
    if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
        raise ValueError("net buffers must be contiguous float32 CUDA tensors")
    if n is not None and t.numel() < n:
        raise ValueError(f"buffer has {t.numel()} entries, needs {n}")
    return ctypes.c_void_p(t.data_ptr())


def _ints(values):
    values = [int(v) for v in np.asarray(values).reshape(-1)]
    return (ctypes.c_int * max(1, len(values)))(*values)


def _host_params(params):
    if params is None:
        return None
    a = np.ascontiguousarray(params, dtype=np.float32).reshape(-1)
    if a.size != GA_GNET_NPARAM:
        raise ValueError(f"need {GA_GNET_NPARAM} parameters")
    return a


class GNet:
    """Learned-guess net (ga_gnet_create); params: host array of GA_GNET_NPARAM floats or None."""

    def __init__(self, params=None):
        lib = load_library()
        a = _host_params(params)
        h = ctypes.c_void_p()
        _check(lib.ga_gnet_create(None if a is None else a.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                  ctypes.byref(h)))
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            _lib.ga_gnet_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def ga_gnet_create(params=None):
    return GNet(params)


def ga_gnet_set_params(net, params):
    a = _host_params(params)
    _check(_lib.ga_gnet_set_params(net.h, a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))


def ga_gnet_get_params(net):
    a = np.zeros(GA_GNET_NPARAM, dtype=np.float32)
    _check(_lib.ga_gnet_get_params(net.h, a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))
    return a


def _hist_array(patch, hist):
    if len(hist) != 4:
        raise ValueError("need 4 history vectors (newest first)")
    return (ctypes.c_void_p * 4)(*[_ptr(h, patch.n_free).value for h in hist])


def ga_gnet_set_train_prec(net, prec):
    _check(_lib.ga_gnet_set_train_prec(net.h, int(prec)))


def ga_gnet_make_batch(net, patch, hist, x, origins, S, inp, tgt):
    nb = len(origins)
    T = S - 6
    _check(_lib.ga_gnet_make_batch(net.h, patch.h, _hist_array(patch, hist), _ptr(x, patch.n_free), nb, int(S),
                                   _ints(origins), _fptr(inp, nb * 4 * S ** 3), _fptr(tgt, nb * T ** 3),
                                   _stream()))


def ga_gnet_forward(net, grid, origins, S, inp, out):
    nb = len(origins)
    _check(_lib.ga_gnet_forward(net.h, nb, int(S), _ints(grid), _ints(origins), _fptr(inp, nb * 4 * S ** 3),
                                _fptr(out, nb * (S - 6) ** 3), _stream()))


def ga_gnet_loss_grad(net, grid, origins, S, inp, tgt, grad, want_loss=True):
    nb = len(origins)
    loss = ctypes.c_double()
    _check(_lib.ga_gnet_loss_grad(net.h, nb, int(S), _ints(grid), _ints(origins), _fptr(inp, nb * 4 * S ** 3),
                                  _fptr(tgt, nb * (S - 6) ** 3), _fptr(grad, GA_GNET_NPARAM),
                                  ctypes.byref(loss) if want_loss else None, _stream()))
    return loss.value if want_loss else None


def ga_gnet_adam(net, grad, lr):
    _check(_lib.ga_gnet_adam(net.h, _fptr(grad, GA_GNET_NPARAM), ctypes.c_float(lr), _stream()))


def ga_gnet_infer(net, patch, hist, x):
    _check(_lib.ga_gnet_infer(net.h, patch.h, _hist_array(patch, hist), _ptr(x, patch.n_free), _stream()))


def ga_integrator_history(integ):
    n = ctypes.c_int()
    _check(_lib.ga_integrator_history(integ.h, ctypes.byref(n)))
    return n.value


def ga_integrator_set_history(integ, hist):
    """hist[age][stage]: device vectors of n_free, age 0 the newest."""
    flat = [h for per_age in hist for h in per_age]
    arr = (ctypes.c_void_p * max(1, len(flat)))(*[_ptr(t, integ.patch.n_free) for t in flat])
    _check(_lib.ga_integrator_set_history(integ.h, len(hist), arr if flat else None, _stream()))


def ga_integrator_set_net(integ, stage, net):
    _check(_lib.ga_integrator_set_net(integ.h, int(stage), None if net is None else net.h))
    # the integrator holds the net's handle: keep the Python object alive with it
    integ.__dict__.setdefault("_nets", {})[int(stage)] = net


# ---- batched independent patches ----

class Batch:
    """R independent 3-D patches stepped together (ga_batch_create)."""

    def __init__(self, patches, k, rho, tau, rtol=1e-10, maxit=200):
        lib = load_library()
        arr = (ctypes.c_void_p * len(patches))(*[p.h.value for p in patches])
        h = ctypes.c_void_p()
        _check(lib.ga_batch_create(len(patches), arr, int(k), float(rho), float(tau), float(rtol), int(maxit),
                                   ctypes.byref(h)))
        self.h, self.patches, self.k = h, list(patches), k
        n = ctypes.c_longlong()
        offs = (ctypes.c_longlong * len(patches))()
        _check(lib.ga_batch_info(h, ctypes.byref(n), offs, None))
        self.n_total, self.offsets = n.value, list(offs)

    def close(self):
        if getattr(self, "h", None):
            _lib.ga_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def ga_batch_create(patches, k, rho, tau, rtol=1e-10, maxit=200):
    return Batch(patches, k, rho, tau, rtol, maxit)


def ga_batch_graph_replays(batch):
    r = ctypes.c_longlong()
    _check(_lib.ga_batch_info(batch.h, None, None, ctypes.byref(r)))
    return r.value


def ga_batch_set_precision(batch, prec):
    """GA_FP64 or GA_FP32 (FP32 inner PCG inside FP64 refinement) mass solves."""
    _check(_lib.ga_batch_set_precision(batch.h, int(prec), _stream()))


def ga_batch_set_tau(batch, taus):
    """Per-patch time steps (None: the common tau of the batch)."""
    if taus is None:
        _check(_lib.ga_batch_set_tau(batch.h, None))
        return
    t = np.ascontiguousarray(np.asarray(taus, dtype=np.float64))
    if len(t) != len(batch.patches):
        raise ValueError("one time step per patch")
    _check(_lib.ga_batch_set_tau(batch.h, t.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))


def ga_batch_tune(batch, reps=5):
    ms = ctypes.c_double()
    _check(_lib.ga_batch_tune(batch.h, int(reps), ctypes.byref(ms), _stream()))
    return ms.value


def _batch_state(batch, state):
    ns = 3 * batch.k
    if len(state) != ns:
        raise ValueError(f"need {ns} state vectors")
    return (ctypes.c_void_p * ns)(*[_ptr(s, batch.n_total).value for s in state])


def ga_batch_init_state(batch, U0, V0, state):
    n = batch.n_total
    _check(_lib.ga_batch_init_state(batch.h, _ptr(U0, n), _ptr(V0, n), _batch_state(batch, state), _stream()))


def ga_batch_step(batch, state, nsteps=1, use_graph=True):
    """Advance; returns int array [nsteps, k, npatch] of PCG iterations."""
    R = len(batch.patches)
    its = (ctypes.c_int * (nsteps * batch.k * R))()
    _check(_lib.ga_batch_step(batch.h, _batch_state(batch, state), int(nsteps), 1 if use_graph else 0, its,
                              _stream()))
    return np.array(its, dtype=np.int64).reshape(nsteps, batch.k, R)


# ---- glued multi-patch domain ----

class MultiPatch:
    """Brick of P[0] x P[1] x P[2] C^0-glued patches (ga_mp_create)."""

    def __init__(self, P, n_el, p, ctrls, k, rho, tau, rtol=1e-10, maxit=200):
        lib = load_library()
        keep = [np.ascontiguousarray(c, dtype=np.float64) for c in ctrls]
        arr = (ctypes.c_void_p * len(keep))(*[c.ctypes.data for c in keep])
        Pa = (ctypes.c_int * 3)(*[int(v) for v in P])
        h = ctypes.c_void_p()
        _check(lib.ga_mp_create(Pa, int(n_el), int(p), arr, int(k), float(rho), float(tau), float(rtol),
                                int(maxit), _stream(), ctypes.byref(h)))
        self.h, self.k = h, k
        n, nl = ctypes.c_longlong(), ctypes.c_longlong()
        mfg = (ctypes.c_int * 3)()
        _check(lib.ga_mp_info(h, ctypes.byref(n), mfg, ctypes.byref(nl)))
        self.n_global, self.mfg, self.n_local = n.value, tuple(mfg), nl.value

    def close(self):
        if getattr(self, "h", None):
            _lib.ga_mp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def ga_mp_create(P, n_el, p, ctrls, k, rho, tau, rtol=1e-10, maxit=200):
    return MultiPatch(P, n_el, p, ctrls, k, rho, tau, rtol, maxit)


def ga_mp_apply(mp, which, x, y, nrhs=1):
    n = nrhs * mp.n_global
    _check(_lib.ga_mp_apply(mp.h, which.encode(), nrhs, _ptr(x, n), _ptr(y, n), _stream()))


def ga_mp_mass_solve(mp, b, x, nrhs=1):
    n = nrhs * mp.n_global
    its = (ctypes.c_int * nrhs)()
    _check(_lib.ga_mp_mass_solve(mp.h, nrhs, _ptr(b, n), _ptr(x, n), its, _stream()))
    return list(its)


def _mp_state(mp, state):
    ns = 3 * mp.k
    if len(state) != ns:
        raise ValueError(f"need {ns} state vectors")
    return (ctypes.c_void_p * ns)(*[_ptr(s, mp.n_global).value for s in state])


def ga_mp_init_state(mp, U0, V0, state):
    n = mp.n_global
    _check(_lib.ga_mp_init_state(mp.h, _ptr(U0, n), _ptr(V0, n), _mp_state(mp, state), _stream()))


def ga_mp_step(mp, state, nsteps=1):
    its = (ctypes.c_int * (nsteps * mp.k))()
    _check(_lib.ga_mp_step(mp.h, _mp_state(mp, state), int(nsteps), its, _stream()))
    return np.array(its, dtype=np.int64).reshape(nsteps, mp.k)


# ---- batched 1-D wave problems (dispersion study) ----

class Wave1D:
    """nsys independent 1-D problems M U'' + omega_r^2 K U = 0 (ga_wave1d_create)."""

    def __init__(self, n_el, p, omega2, k, rho_b, rho_s, tau):
        lib = load_library()
        w2 = np.ascontiguousarray(np.asarray(omega2, dtype=np.float64))
        h = ctypes.c_void_p()
        _check(lib.ga_wave1d_create(int(n_el), int(p), len(w2), w2.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                    int(k), float(rho_b), float(rho_s), float(tau), ctypes.byref(h)))
        self.h, self.k, self.nsys = h, int(k), len(w2)
        m = ctypes.c_int()
        _check(lib.ga_wave1d_info(h, ctypes.byref(m)))
        self.m = m.value
        self.n_total = self.nsys * self.m

    def close(self):
        if getattr(self, "h", None):
            _lib.ga_wave1d_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _w1_state(w, state):
    if len(state) != 3 * w.k:
        raise ValueError(f"need {3 * w.k} state vectors")
    return (ctypes.c_void_p * len(state))(*[_ptr(s, w.n_total).value for s in state])


def ga_wave1d_load_sine(w, wavenumbers, f):
    j = np.ascontiguousarray(np.asarray(wavenumbers, dtype=np.float64))
    if len(j) != w.nsys:
        raise ValueError("one wavenumber per system")
    _check(_lib.ga_wave1d_load_sine(w.h, j.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                    _ptr(f, w.n_total), _stream()))


def ga_wave1d_apply(w, which, x, y):
    _check(_lib.ga_wave1d_apply(w.h, which.encode()[:1], _ptr(x, w.n_total), _ptr(y, w.n_total), _stream()))


def ga_wave1d_init_state(w, U0, V0, state):
    _check(_lib.ga_wave1d_init_state(w.h, _ptr(U0, w.n_total), _ptr(V0, w.n_total), _w1_state(w, state),
                                     _stream()))


def ga_wave1d_step(w, state, nsteps=1):
    _check(_lib.ga_wave1d_step(w.h, _w1_state(w, state), int(nsteps), _stream()))

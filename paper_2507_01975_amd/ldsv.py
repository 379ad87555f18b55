"""ctypes binding of libldsv.so (argument marshalling only).

Every function takes torch tensors that already live on the GPU, checks
their dtype, shape and contiguity, and passes raw device pointers and the
current HIP stream to the C ABI declared in include/ldsv.h.  No numerical
step runs here.  If the shared library is missing the import fails loudly:
there is no CPU fallback.
"""
import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "lib", "libldsv.so")

OK, EINVAL, ESHAPE, EDTYPE, EHIP, ENONFINITE, ENOMEM = 0, -1, -2, -3, -4, -5, -6
F32, F64 = 0, 1
MAC, COLLOCATED = 0, 1
RK4, SSPRK3 = 0, 1
ADVECTION, VISCOSITY, FORCING, ALL_PHYSICS = 1, 2, 4, 7
IC_FOURIER_MODES, IC_GRF_PEAK, IC_TGV, IC_SHEAR_LAYER = 0, 1, 2, 3
NCOEF, NOUT, NLAYERS = 64, 66, 6
# (C_in, C_out) of the coefficient network's six 3x3 layers, as ldsv_net lays
# them out: 2 -> 64 -> 64 -> 64 -> 64 -> 64 -> 66
LAYERS = [(2, 64)] + [(64, 64)] * (NLAYERS - 2) + [(64, NOUT)]


class LdsvError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("ldsv error %d: %s" % (code, msg))
        self.code = code


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError("libldsv.so is not built (%s); run `python -m paper_2507_01975_amd.build`"
                          % LIB_PATH)
    return ctypes.CDLL(LIB_PATH)


_lib = _load()


class Grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("lx", ctypes.c_double),
                ("ly", ctypes.c_double), ("batch", ctypes.c_int), ("dtype", ctypes.c_int),
                ("layout", ctypes.c_int)]


class Params(ctypes.Structure):
    _fields_ = [("nu", ctypes.c_double), ("forcing_amp", ctypes.c_double),
                ("forcing_k", ctypes.c_double), ("drag", ctypes.c_double),
                ("dt", ctypes.c_double), ("rk", ctypes.c_int), ("physics_mask", ctypes.c_int),
                ("k_c", ctypes.c_int), ("guard_threshold", ctypes.c_double),
                ("fallback_enable", ctypes.c_int)]


class ICArgs(ctypes.Structure):
    _fields_ = [("amp", ctypes.c_double), ("k", ctypes.c_double), ("delta", ctypes.c_double),
                ("pert", ctypes.c_double), ("noise_rms", ctypes.c_double),
                ("kpeak", ctypes.c_double)]


class Net(ctypes.Structure):
    _fields_ = [("w", ctypes.c_void_p * NLAYERS), ("b", ctypes.c_void_p * NLAYERS)]


class NetGrad(ctypes.Structure):
    _fields_ = [("w", ctypes.c_void_p * NLAYERS), ("b", ctypes.c_void_p * NLAYERS)]


class Fno(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int), ("layers", ctypes.c_int), ("modes", ctypes.c_int),
                ("n_in", ctypes.c_int), ("n_out", ctypes.c_int), ("lift_w", ctypes.c_void_p), ("lift_b", ctypes.c_void_p),
                ("spec_w", ctypes.c_void_p), ("point_w", ctypes.c_void_p),
                ("point_b", ctypes.c_void_p), ("proj_w", ctypes.c_void_p),
                ("proj_b", ctypes.c_void_p)]


class FluxNet(ctypes.Structure):
    _fields_ = [("stencil_w", ctypes.c_void_p), ("fno", ctypes.POINTER(Fno) * 2)]


class FnoGrad(ctypes.Structure):
    _fields_ = [("lift_w", ctypes.c_void_p), ("lift_b", ctypes.c_void_p),
                ("spec_w", ctypes.c_void_p), ("point_w", ctypes.c_void_p),
                ("point_b", ctypes.c_void_p), ("proj_w", ctypes.c_void_p),
                ("proj_b", ctypes.c_void_p)]


class FluxNetGrad(ctypes.Structure):
    _fields_ = [("stencil_w", ctypes.c_void_p), ("fno", ctypes.POINTER(FnoGrad) * 2)]


_vp = ctypes.c_void_p
_i = ctypes.c_int
_d = ctypes.c_double
_sz = ctypes.c_size_t

_SIGS = {
    "ldsv_version": ([], _i),
    "ldsv_last_error": ([], ctypes.c_char_p),
    "ldsv_create": ([ctypes.POINTER(_vp), ctypes.POINTER(Grid)], _i),
    "ldsv_destroy": ([_vp], _i),
    "ldsv_workspace_bytes": ([_vp, ctypes.POINTER(_sz)], _i),
    "ldsv_init_state": ([_vp, _i, ctypes.c_uint64, ctypes.POINTER(ICArgs), _vp, _vp, _vp], _i),
    "ldsv_rhs": ([_vp, ctypes.POINTER(Params), _vp, _vp, _vp, _vp, _vp, _vp], _i),
    "ldsv_fv_step": ([_vp, ctypes.POINTER(Params), _vp, _vp, _vp, _vp, _vp, _i, _vp], _i),
    "ldsv_fv_step_noalloc": ([ctypes.POINTER(Grid), ctypes.POINTER(Params), _vp, _vp, _vp, _vp,
                              _vp, _i, _vp], _i),
    "ldsv_project": ([_vp, _vp, _vp, _vp, _vp], _i),
    "ldsv_project_bwd": ([_vp, _vp, _vp, _vp], _i),
    "ldsv_cnn_forward": ([_vp, ctypes.POINTER(Net), _vp, _vp, _vp, _vp], _i),
    "ldsv_cnn_activation": ([_vp, _i, _vp, _vp], _i),
    "ldsv_learned_fv_step": ([_vp, ctypes.POINTER(Params), ctypes.POINTER(Net), _vp, _vp, _vp,
                              _vp, _i, _vp, _vp], _i),
    "ldsv_rollout": ([_vp, ctypes.POINTER(Params), ctypes.POINTER(Net), _vp, _vp, _i, _i, _i,
                      _vp, _vp, _vp, _vp], _i),
    "ldsv_fv_step_bwd": ([_vp, ctypes.POINTER(Params), _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                          _vp], _i),
    "ldsv_cnn_backward": ([_vp, ctypes.POINTER(Net), _vp, _vp, _vp, _vp, _vp,
                           ctypes.POINTER(NetGrad), _vp], _i),
    "ldsv_learned_fv_step_bwd": ([_vp, ctypes.POINTER(Params), ctypes.POINTER(Net), _vp, _vp, _i,
                                  _vp, _vp, _vp, _vp, ctypes.POINTER(NetGrad), _vp], _i),
    "ldsv_rollout_bwd": ([_vp, ctypes.POINTER(Params), ctypes.POINTER(Net), _vp, _vp, _i, _i, _i,
                          _vp, _vp, _d, _vp, _vp, _vp, _vp, ctypes.POINTER(NetGrad), _vp, _vp], _i),
    "ldsv_fv_step_d": ([_vp, ctypes.POINTER(Params), _vp, _vp, _vp, _vp, _vp, _vp, _i, _vp], _i),
    "ldsv_fv_step_d_bwd": ([_vp, ctypes.POINTER(Params), _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                            _vp, _vp, _vp], _i),
    "ldsv_learned_d_fv_step": ([_vp, ctypes.POINTER(Params), ctypes.POINTER(Net),
                                ctypes.POINTER(Net), _vp, _vp, _vp, _vp, _i, _vp, _vp, _vp], _i),
    "ldsv_learned_d_fv_step_bwd": ([_vp, ctypes.POINTER(Params), ctypes.POINTER(Net),
                                    ctypes.POINTER(Net), _vp, _vp, _i, _vp, _vp, _vp, _vp,
                                    ctypes.POINTER(NetGrad), ctypes.POINTER(NetGrad), _vp], _i),
    "ldsv_rollout_d": ([_vp, ctypes.POINTER(Params), ctypes.POINTER(Net), ctypes.POINTER(Net),
                        _vp, _vp, _i, _i, _i, _vp, _vp, _vp, _vp], _i),
    "ldsv_rollout_d_bwd": ([_vp, ctypes.POINTER(Params), ctypes.POINTER(Net), ctypes.POINTER(Net),
                            _vp, _vp, _i, _i, _i, _vp, _vp, _d, _vp, _vp, _vp, _vp,
                            ctypes.POINTER(NetGrad), ctypes.POINTER(NetGrad), _vp, _vp], _i),
    "ldsv_mse_grad": ([_vp, _vp, _vp, _vp, _vp, _d, _vp, _vp, _vp, _vp], _i),
    "ldsv_adam_step": ([_vp, _vp, _vp, _vp, _sz, _i, _d, _d, _d, _d, _vp], _i),
    "ldsv_to_bf16": ([_vp, _vp, _sz, _vp], _i),
    "ldsv_downsample": ([_vp, _i, _vp, _vp, _vp, _vp, _vp], _i),
    "ldsv_vorticity": ([_vp, _vp, _vp, _vp, _vp], _i),
    "ldsv_pcc": ([_vp, _vp, _vp, _vp, _vp], _i),
    "ldsv_diagnostics": ([_vp, _vp, _vp, _vp, _vp], _i),
    "ldsv_cfl_dt": ([_vp, _vp, _vp, _d, ctypes.POINTER(_d), _vp], _i),
    "ldsv_fno_forward": ([_vp, ctypes.POINTER(FluxNet), _vp, _vp, _vp, _vp], _i),
    "ldsv_fluxblock_fv_step": ([_vp, ctypes.POINTER(Params), _vp, _vp, _vp, _vp, _vp, _vp, _i,
                                _vp], _i),
    "ldsv_fluxblock_fv_step_bwd": ([_vp, ctypes.POINTER(Params), _vp, _vp, _vp, _vp, _vp, _vp,
                                    _vp, _vp, _vp, _vp, _vp], _i),
    "ldsv_fluxblock_step": ([_vp, ctypes.POINTER(Params), ctypes.POINTER(FluxNet), _vp, _vp, _vp,
                             _vp, _vp, _vp], _i),
    "ldsv_fno_backward": ([_vp, ctypes.POINTER(FluxNet), _vp, _vp, _vp, _vp, _vp,
                           ctypes.POINTER(FluxNetGrad), _vp], _i),
    "ldsv_fluxblock_step_bwd": ([_vp, ctypes.POINTER(Params), ctypes.POINTER(FluxNet), _vp, _vp,
                                 _vp, _vp, _vp, _vp, ctypes.POINTER(FluxNetGrad), _vp], _i),
    "ldsv_fluxblock_tc_step": ([_vp, ctypes.POINTER(Params), ctypes.POINTER(FluxNet),
                                ctypes.POINTER(Fno), ctypes.POINTER(_vp), ctypes.POINTER(_vp), _i,
                                _vp, _vp, _vp], _i),
    "ldsv_fluxblock_tc_step_bwd": ([_vp, ctypes.POINTER(Params), ctypes.POINTER(FluxNet),
                                    ctypes.POINTER(Fno), ctypes.POINTER(_vp), ctypes.POINTER(_vp),
                                    _i, _vp, _vp, ctypes.POINTER(_vp), ctypes.POINTER(_vp),
                                    ctypes.POINTER(FluxNetGrad), ctypes.POINTER(FnoGrad), _vp],
                                   _i),
    "ldsv_fv_step_scalar": ([_vp, ctypes.POINTER(Params), _d, _vp, _vp, _vp, _vp, _vp, _vp, _i,
                             _vp], _i),
    "ldsv_init_scalar": ([_vp, ctypes.POINTER(ICArgs), _vp, _vp], _i),
    "ldsv_timer_enable": ([_vp, _i], _i),
    "ldsv_timer_read": ([_vp, _i, ctypes.POINTER(_d), ctypes.POINTER(_i)], _i),
}

# kernel classes of ldsv_timer_read
TIMER_STAGE, TIMER_ROWFFT, TIMER_COLSOLVE, TIMER_ROWIFFT, TIMER_CONV, TIMER_CONV0, TIMER_ADJ, \
    TIMER_OTHER, TIMER_FNO_FFT, TIMER_FNO_MIX = range(10)

for _name, (_args, _res) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = _res


def exported_symbols():
    return list(_SIGS)


def last_error():
    return _lib.ldsv_last_error().decode()


def _check(rc):
    if rc != OK:
        raise LdsvError(rc, last_error())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    if t is None:
        return None
    return ctypes.c_void_p(t.data_ptr())


class Solver:
    """A handle for one grid: nx x ny cells, `batch` trajectories."""

    def __init__(self, nx, ny, batch, lx=2 * 3.141592653589793, ly=2 * 3.141592653589793,
                 dtype=torch.float32, layout=MAC):
        self.nx, self.ny, self.batch = nx, ny, batch
        self.lx, self.ly = lx, ly
        self.dtype = dtype
        self.layout = layout
        g = Grid(nx, ny, lx, ly, batch, F64 if dtype == torch.float64 else F32, layout)
        h = ctypes.c_void_p()
        _check(_lib.ldsv_create(ctypes.byref(h), ctypes.byref(g)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            _lib.ldsv_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- tensor checks
    def _state(self, t, name="state", dtype=None):
        dt = dtype or self.dtype
        if not (t.is_cuda and t.dtype == dt and t.is_contiguous()
                and tuple(t.shape) == (self.batch, self.ny, self.nx)):
            raise ValueError("%s must be a contiguous %s cuda tensor of shape %s, got %s %s %s"
                             % (name, dt, (self.batch, self.ny, self.nx), t.dtype,
                                tuple(t.shape), t.device))
        return _ptr(t)

    def new_state(self):
        return torch.empty(self.batch, self.ny, self.nx, dtype=self.dtype, device="cuda")

    def workspace_bytes(self):
        b = ctypes.c_size_t()
        _check(_lib.ldsv_workspace_bytes(self._h, ctypes.byref(b)))
        return b.value

    # ---- calls
    def init_state(self, kind, seed, u=None, v=None, **kw):
        u = self.new_state() if u is None else u
        v = self.new_state() if v is None else v
        ic = None
        if kw:
            base = dict(amp=1.0, k=1.0, delta=1.0 / 30.0, pert=0.05, noise_rms=1e-3, kpeak=4.0)
            base.update(kw)
            ic = ctypes.byref(ICArgs(**base))
        _check(_lib.ldsv_init_state(self._h, kind, seed, ic, self._state(u), self._state(v),
                                    _stream()))
        return u, v

    def rhs(self, prm, u, v, coef=None):
        ru, rv = self.new_state(), self.new_state()
        _check(_lib.ldsv_rhs(self._h, ctypes.byref(prm), self._coef(coef), self._state(u),
                             self._state(v), _ptr(ru), _ptr(rv), _stream()))
        return ru, rv

    def _coef(self, coef):
        if coef is None:
            return None
        if not (coef.is_cuda and coef.dtype == torch.float32 and coef.is_contiguous()
                and tuple(coef.shape) == (self.batch, NCOEF, self.ny, self.nx)):
            raise ValueError("coef must be float32 [B, 64, Ny, Nx] contiguous on cuda")
        return _ptr(coef)

    def fv_step(self, prm, u, v, nsteps=1, coef=None, out=None):
        uo, vo = (self.new_state(), self.new_state()) if out is None else out
        _check(_lib.ldsv_fv_step(self._h, ctypes.byref(prm), self._coef(coef), self._state(u),
                                 self._state(v), self._state(uo), self._state(vo), nsteps,
                                 _stream()))
        return uo, vo

    def project(self, u, v, want_p=False):
        """In place; returns p if want_p."""
        p = self.new_state() if want_p else None
        _check(_lib.ldsv_project(self._h, self._state(u), self._state(v), _ptr(p), _stream()))
        return p

    def project_bwd(self, gu, gv):
        _check(_lib.ldsv_project_bwd(self._h, self._state(gu), self._state(gv), _stream()))

    def cnn_forward(self, net, u, v):
        out = torch.empty(self.batch, NOUT, self.ny, self.nx, dtype=torch.float32, device="cuda")
        _check(_lib.ldsv_cnn_forward(self._h, ctypes.byref(net.c), self._state(u),
                                     self._state(v), _ptr(out), _stream()))
        return out

    def cnn_activation(self, layer):
        """bf16 NHWC activation of layer 0..4 from the last network pass, as
        float32 [B, 64, Ny, Nx]."""
        a = torch.empty(self.batch, self.ny, self.nx, 64, dtype=torch.int16, device="cuda")
        _check(_lib.ldsv_cnn_activation(self._h, layer, _ptr(a), _stream()))
        return a.view(torch.bfloat16).float().permute(0, 3, 1, 2).contiguous()

    def learned_fv_step(self, prm, net, u, v, step_index, want_net_out=False, out=None):
        uo, vo = (self.new_state(), self.new_state()) if out is None else out
        no = None
        if want_net_out:
            no = torch.empty(self.batch, NOUT, self.ny, self.nx, dtype=torch.float32,
                             device="cuda")
        _check(_lib.ldsv_learned_fv_step(self._h, ctypes.byref(prm), ctypes.byref(net.c),
                                         self._state(u), self._state(v), self._state(uo),
                                         self._state(vo), step_index, _ptr(no), _stream()))
        return (uo, vo, no) if want_net_out else (uo, vo)

    def rollout(self, prm, u0, v0, nsteps, save_every=1, net=None, first_index=1,
                fallback_flags=None):
        T = nsteps // save_every
        tu = torch.empty(T, self.batch, self.ny, self.nx, dtype=self.dtype, device="cuda")
        tv = torch.empty_like(tu)
        _check(_lib.ldsv_rollout(self._h, ctypes.byref(prm),
                                 ctypes.byref(net.c) if net is not None else None,
                                 self._state(u0), self._state(v0), nsteps, save_every,
                                 first_index, _ptr(tu), _ptr(tv), _ptr(fallback_flags), _stream()))
        return tu, tv

    def fv_step_bwd(self, prm, u, v, gu_out, gv_out, coef=None, gcoef=None):
        gu, gv = self.new_state(), self.new_state()
        _check(_lib.ldsv_fv_step_bwd(self._h, ctypes.byref(prm), self._coef(coef),
                                     self._state(u), self._state(v), self._state(gu_out),
                                     self._state(gv_out), _ptr(gu), _ptr(gv),
                                     self._coef(gcoef), _stream()))
        return gu, gv

    def cnn_backward(self, net, u, v, gout, dW, want_input_grad=True):
        gu = self.new_state() if want_input_grad else None
        gv = self.new_state() if want_input_grad else None
        _check(_lib.ldsv_cnn_backward(self._h, ctypes.byref(net.c), self._state(u),
                                      self._state(v), _ptr(gout.contiguous()), _ptr(gu), _ptr(gv),
                                      ctypes.byref(dW.c), _stream()))
        return gu, gv

    def learned_fv_step_bwd(self, prm, net, u, v, step_index, gu_out, gv_out, dW):
        gu, gv = self.new_state(), self.new_state()
        _check(_lib.ldsv_learned_fv_step_bwd(self._h, ctypes.byref(prm), ctypes.byref(net.c),
                                             self._state(u), self._state(v), step_index,
                                             self._state(gu_out), self._state(gv_out), _ptr(gu),
                                             _ptr(gv), ctypes.byref(dW.c), _stream()))
        return gu, gv

    def rollout_bwd(self, prm, net, u0, v0, nsteps, dW, checkpoint_every=8, first_index=1,
                    labels=None, loss_scale=1.0, g_traj=None, want_input_grad=False, loss=None):
        """Unrolled backward with checkpoints; returns (gu0, gv0) or None."""
        lu = lv = gtu = gtv = None
        if labels is not None:
            lu, lv = labels
            for t in (lu, lv):
                if tuple(t.shape) != (nsteps, self.batch, self.ny, self.nx) or not t.is_contiguous():
                    raise ValueError("labels must be contiguous [nsteps, B, Ny, Nx]")
        if g_traj is not None:
            gtu, gtv = g_traj
        gu = self.new_state() if want_input_grad else None
        gv = self.new_state() if want_input_grad else None
        _check(_lib.ldsv_rollout_bwd(self._h, ctypes.byref(prm), ctypes.byref(net.c),
                                     self._state(u0), self._state(v0), nsteps, checkpoint_every,
                                     first_index, _ptr(lu), _ptr(lv), loss_scale, _ptr(gtu),
                                     _ptr(gtv), _ptr(gu), _ptr(gv), ctypes.byref(dW.c), _ptr(loss),
                                     _stream()))
        return (gu, gv) if want_input_grad else None

    # ---- learned derivative stencils (per cell; a second network dnet) ----

    def fv_step_d(self, prm, u, v, coef, dcoef, nsteps=1, out=None):
        uo, vo = (self.new_state(), self.new_state()) if out is None else out
        _check(_lib.ldsv_fv_step_d(self._h, ctypes.byref(prm), self._coef(coef), self._coef(dcoef),
                                   self._state(u), self._state(v), self._state(uo),
                                   self._state(vo), nsteps, _stream()))
        return uo, vo

    def fv_step_d_bwd(self, prm, u, v, gu_out, gv_out, coef, dcoef, gcoef=None, gdcoef=None):
        gu, gv = self.new_state(), self.new_state()
        _check(_lib.ldsv_fv_step_d_bwd(self._h, ctypes.byref(prm), self._coef(coef),
                                       self._coef(dcoef), self._state(u), self._state(v),
                                       self._state(gu_out), self._state(gv_out), _ptr(gu),
                                       _ptr(gv), self._coef(gcoef), self._coef(gdcoef),
                                       _stream()))
        return gu, gv

    def learned_d_fv_step(self, prm, net, dnet, u, v, step_index, want_net_out=False, out=None):
        uo, vo = (self.new_state(), self.new_state()) if out is None else out
        no = dno = None
        if want_net_out:
            no = torch.empty(self.batch, NOUT, self.ny, self.nx, dtype=torch.float32,
                             device="cuda")
            dno = torch.empty_like(no)
        _check(_lib.ldsv_learned_d_fv_step(self._h, ctypes.byref(prm), ctypes.byref(net.c),
                                           ctypes.byref(dnet.c), self._state(u), self._state(v),
                                           self._state(uo), self._state(vo), step_index, _ptr(no),
                                           _ptr(dno), _stream()))
        return (uo, vo, no, dno) if want_net_out else (uo, vo)

    def learned_d_fv_step_bwd(self, prm, net, dnet, u, v, step_index, gu_out, gv_out, dW, dWd):
        gu, gv = self.new_state(), self.new_state()
        _check(_lib.ldsv_learned_d_fv_step_bwd(self._h, ctypes.byref(prm), ctypes.byref(net.c),
                                               ctypes.byref(dnet.c), self._state(u),
                                               self._state(v), step_index, self._state(gu_out),
                                               self._state(gv_out), _ptr(gu), _ptr(gv),
                                               ctypes.byref(dW.c), ctypes.byref(dWd.c),
                                               _stream()))
        return gu, gv

    def rollout_d(self, prm, net, dnet, u0, v0, nsteps, save_every=1, first_index=1,
                  fallback_flags=None):
        T = nsteps // save_every
        tu = torch.empty(T, self.batch, self.ny, self.nx, dtype=self.dtype, device="cuda")
        tv = torch.empty_like(tu)
        _check(_lib.ldsv_rollout_d(self._h, ctypes.byref(prm), ctypes.byref(net.c),
                                   ctypes.byref(dnet.c), self._state(u0), self._state(v0), nsteps,
                                   save_every, first_index, _ptr(tu), _ptr(tv),
                                   _ptr(fallback_flags), _stream()))
        return tu, tv

    def rollout_d_bwd(self, prm, net, dnet, u0, v0, nsteps, dW, dWd, checkpoint_every=8,
                      first_index=1, labels=None, loss_scale=1.0, g_traj=None,
                      want_input_grad=False, loss=None):
        lu = lv = gtu = gtv = None
        if labels is not None:
            lu, lv = labels
            for t in (lu, lv):
                if tuple(t.shape) != (nsteps, self.batch, self.ny, self.nx) or not t.is_contiguous():
                    raise ValueError("labels must be contiguous [nsteps, B, Ny, Nx]")
        if g_traj is not None:
            gtu, gtv = g_traj
        gu = self.new_state() if want_input_grad else None
        gv = self.new_state() if want_input_grad else None
        _check(_lib.ldsv_rollout_d_bwd(self._h, ctypes.byref(prm), ctypes.byref(net.c),
                                       ctypes.byref(dnet.c), self._state(u0), self._state(v0),
                                       nsteps, checkpoint_every, first_index, _ptr(lu), _ptr(lv),
                                       loss_scale, _ptr(gtu), _ptr(gtv), _ptr(gu), _ptr(gv),
                                       ctypes.byref(dW.c), ctypes.byref(dWd.c), _ptr(loss),
                                       _stream()))
        return (gu, gv) if want_input_grad else None

    def mse_grad(self, u, v, lu, lv, scale=1.0, loss=None, want_grad=True):
        gu = self.new_state() if want_grad else None
        gv = self.new_state() if want_grad else None
        _check(_lib.ldsv_mse_grad(self._h, self._state(u), self._state(v), self._state(lu),
                                  self._state(lv), scale, _ptr(gu), _ptr(gv), _ptr(loss),
                                  _stream()))
        return gu, gv

    def downsample(self, r, uf, vf):
        uc, vc = self.new_state(), self.new_state()
        shape = (self.batch, self.ny * r, self.nx * r)
        for t in (uf, vf):
            if tuple(t.shape) != shape or not t.is_contiguous() or t.dtype != self.dtype:
                raise ValueError("fine field must be %s contiguous %s" % (shape, self.dtype))
        _check(_lib.ldsv_downsample(self._h, r, _ptr(uf), _ptr(vf), _ptr(uc), _ptr(vc),
                                    _stream()))
        return uc, vc

    def vorticity(self, u, v):
        w = self.new_state()
        _check(_lib.ldsv_vorticity(self._h, self._state(u), self._state(v), _ptr(w), _stream()))
        return w

    def pcc(self, a, b):
        out = torch.empty(self.batch, dtype=torch.float64, device="cuda")
        _check(_lib.ldsv_pcc(self._h, self._state(a), self._state(b), _ptr(out), _stream()))
        return out

    def diagnostics(self, u, v):
        out = torch.empty(self.batch, 6, dtype=torch.float64, device="cuda")
        _check(_lib.ldsv_diagnostics(self._h, self._state(u), self._state(v), _ptr(out),
                                     _stream()))
        return out

    # ---- shear flow with a passive scalar
    def fv_step_scalar(self, prm, diffusivity, u, v, s, nsteps=1, out=None):
        uo, vo, so = (self.new_state(), self.new_state(), self.new_state()) if out is None else out
        _check(_lib.ldsv_fv_step_scalar(self._h, ctypes.byref(prm), diffusivity, self._state(u),
                                        self._state(v), self._state(s), self._state(uo),
                                        self._state(vo), self._state(so), nsteps, _stream()))
        return uo, vo, so

    def init_scalar(self, delta=1.0 / 30.0, s=None):
        s = self.new_state() if s is None else s
        ic = ICArgs(1.0, 1.0, delta, 0.05, 1e-3, 4.0)
        _check(_lib.ldsv_init_scalar(self._h, ctypes.byref(ic), self._state(s), _stream()))
        return s

    # ---- the paper's flux block (O_P + O_L + O_F)
    def _fields(self, f, name="fields"):
        if f is None:
            return None
        if not (f.is_cuda and f.dtype == torch.float32 and f.is_contiguous()
                and tuple(f.shape) == (self.batch, 8, self.ny, self.nx)):
            raise ValueError("%s must be float32 [B, 8, Ny, Nx] contiguous on cuda" % name)
        return _ptr(f)

    @staticmethod
    def _stencil(w, name="stencil_w"):
        if w is None:
            return None
        if not (w.is_cuda and w.dtype == torch.float32 and w.is_contiguous() and w.numel() == 160):
            raise ValueError("%s must be float32 [2, 4, 20] contiguous on cuda" % name)
        return _ptr(w)

    def fno_forward(self, net, u, v):
        out = torch.empty(self.batch, 8, self.ny, self.nx, dtype=torch.float32, device="cuda")
        _check(_lib.ldsv_fno_forward(self._h, ctypes.byref(net.c), self._state(u),
                                     self._state(v), _ptr(out), _stream()))
        return out

    def fluxblock_fv_step(self, prm, stencil_w, fields, u, v, nsteps=1, out=None):
        uo, vo = (self.new_state(), self.new_state()) if out is None else out
        _check(_lib.ldsv_fluxblock_fv_step(self._h, ctypes.byref(prm), self._stencil(stencil_w),
                                           self._fields(fields), self._state(u), self._state(v),
                                           self._state(uo), self._state(vo), nsteps, _stream()))
        return uo, vo

    def fluxblock_fv_step_bwd(self, prm, stencil_w, fields, u, v, gu_out, gv_out, gstencil=None,
                              gfields=None):
        gu, gv = self.new_state(), self.new_state()
        _check(_lib.ldsv_fluxblock_fv_step_bwd(
            self._h, ctypes.byref(prm), self._stencil(stencil_w), self._fields(fields),
            self._state(u), self._state(v), self._state(gu_out), self._state(gv_out), _ptr(gu),
            _ptr(gv), self._stencil(gstencil, "gstencil"), self._fields(gfields, "gfields"),
            _stream()))
        return gu, gv

    def fluxblock_step(self, prm, net, u, v, want_fields=False, out=None):
        uo, vo = (self.new_state(), self.new_state()) if out is None else out
        f = None
        if want_fields:
            f = torch.empty(self.batch, 8, self.ny, self.nx, dtype=torch.float32, device="cuda")
        _check(_lib.ldsv_fluxblock_step(self._h, ctypes.byref(prm), ctypes.byref(net.c),
                                        self._state(u), self._state(v), self._state(uo),
                                        self._state(vo), _ptr(f), _stream()))
        return (uo, vo, f) if want_fields else (uo, vo)

    def fno_backward(self, net, u, v, gfields, grad, want_input_grad=True):
        gu = self.new_state() if want_input_grad else None
        gv = self.new_state() if want_input_grad else None
        _check(_lib.ldsv_fno_backward(self._h, ctypes.byref(net.c), self._state(u), self._state(v),
                                      self._fields(gfields, "gfields"), _ptr(gu), _ptr(gv),
                                      ctypes.byref(grad.c), _stream()))
        return gu, gv

    def fluxblock_step_bwd(self, prm, net, u, v, gu_out, gv_out, grad):
        gu, gv = self.new_state(), self.new_state()
        _check(_lib.ldsv_fluxblock_step_bwd(self._h, ctypes.byref(prm), ctypes.byref(net.c),
                                            self._state(u), self._state(v), self._state(gu_out),
                                            self._state(gv_out), _ptr(gu), _ptr(gv),
                                            ctypes.byref(grad.c), _stream()))
        return gu, gv

    def _hist(self, states, name):
        for t in states:
            self._state(t, name)
        return (_vp * len(states))(*[t.data_ptr() for t in states])

    def fluxblock_tc_step(self, prm, net, tc, hist_u, hist_v, step_index, out=None):
        """One step of the complete model; hist_u/hist_v: the k_c = prm.k_c
        states u_{k-k_c} .. u_{k-1} (oldest first)."""
        if len(hist_u) != prm.k_c or len(hist_v) != prm.k_c:
            raise ValueError("the history must hold k_c = %d states" % prm.k_c)
        uo, vo = (self.new_state(), self.new_state()) if out is None else out
        _check(_lib.ldsv_fluxblock_tc_step(self._h, ctypes.byref(prm), ctypes.byref(net.c),
                                           ctypes.byref(tc.c) if tc is not None else None,
                                           self._hist(hist_u, "hist_u"),
                                           self._hist(hist_v, "hist_v"), step_index,
                                           self._state(uo), self._state(vo), _stream()))
        return uo, vo

    def fluxblock_tc_step_bwd(self, prm, net, tc, hist_u, hist_v, step_index, gu_out, gv_out,
                              ghist_u, ghist_v, grad, gtc=None):
        """Accumulates into ghist_u/ghist_v (lists like hist_u), grad and gtc."""
        if not (len(hist_u) == len(hist_v) == len(ghist_u) == len(ghist_v) == prm.k_c):
            raise ValueError("the history and its gradients must hold k_c = %d states" % prm.k_c)
        _check(_lib.ldsv_fluxblock_tc_step_bwd(
            self._h, ctypes.byref(prm), ctypes.byref(net.c),
            ctypes.byref(tc.c) if tc is not None else None, self._hist(hist_u, "hist_u"),
            self._hist(hist_v, "hist_v"), step_index, self._state(gu_out), self._state(gv_out),
            self._hist(ghist_u, "ghist_u"), self._hist(ghist_v, "ghist_v"), ctypes.byref(grad.c),
            ctypes.byref(gtc.c) if gtc is not None else None, _stream()))

    def timer_enable(self, on=True):
        _check(_lib.ldsv_timer_enable(self._h, 1 if on else 0))

    def timer_read(self, cls):
        """(total ms, launch count) of kernel class `cls` since timer_enable."""
        t = ctypes.c_double()
        n = ctypes.c_int()
        _check(_lib.ldsv_timer_read(self._h, cls, ctypes.byref(t), ctypes.byref(n)))
        return t.value, n.value

    def cfl_dt(self, u, v, cfl):
        d = ctypes.c_double()
        _check(_lib.ldsv_cfl_dt(self._h, self._state(u), self._state(v), cfl, ctypes.byref(d),
                                _stream()))
        return d.value


def params(nu=0.0, dt=0.0, forcing_amp=0.0, forcing_k=0.0, drag=0.0, rk=RK4,
           mask=ALL_PHYSICS, k_c=1, guard_threshold=0.0, fallback_enable=1):
    return Params(nu, forcing_amp, forcing_k, drag, dt, rk, mask, k_c, guard_threshold,
                  fallback_enable)


class NetParams:
    """Device copies of the coefficient network: bf16 weights [Cout][3][3][Cin]
    (bit patterns in int16 tensors) and float biases, plus an FP32 master
    copy of the weights in the same layout for training."""

    def __init__(self, weights, biases):
        """weights: list of [Cout, Cin, 3, 3] tensors (any float dtype, any
        device); biases: list of [Cout]."""
        self.master_w = [w.detach().to("cuda", torch.float32).permute(0, 2, 3, 1).contiguous()
                         for w in weights]
        self.b = [b.detach().to("cuda", torch.float32).contiguous() for b in biases]
        self.w = [torch.empty(w.shape, dtype=torch.int16, device="cuda") for w in self.master_w]
        self.c = Net()
        self.refresh()

    def refresh(self):
        """Round the master weights to bf16 into the device copies."""
        for l in range(NLAYERS):
            _check(_lib.ldsv_to_bf16(_ptr(self.master_w[l]), _ptr(self.w[l]),
                                     self.master_w[l].numel(), _stream()))
            self.c.w[l] = self.w[l].data_ptr()
            self.c.b[l] = self.b[l].data_ptr()

    def torch_weights(self):
        """Master weights back in [Cout, Cin, 3, 3] order."""
        return [w.permute(0, 3, 1, 2).contiguous() for w in self.master_w]

    def bf16_weights(self):
        return [w.view(torch.bfloat16).float().permute(0, 3, 1, 2).contiguous() for w in self.w]


class NetGradBuffers:
    def __init__(self, net):
        self.w = [torch.zeros_like(w) for w in net.master_w]
        self.b = [torch.zeros_like(b) for b in net.b]
        self.c = NetGrad()
        for l in range(NLAYERS):
            self.c.w[l] = self.w[l].data_ptr()
            self.c.b[l] = self.b[l].data_ptr()

    def zero_(self):
        for t in self.w + self.b:
            t.zero_()


NOALLOC_SCRATCH_BYTES = 32 << 20


def fv_step_noalloc(prm, u, v, nsteps=1, coef=None, out=None, lx=2 * 3.141592653589793,
                    ly=2 * 3.141592653589793, layout=MAC):
    """ldsv_fv_step without a handle: the workspace is the library's fixed
    device scratch array, nothing is allocated by the library (outputs are
    allocated here only when `out` is None).  u, v: [B, Ny, Nx] float32 or
    float64 cuda tensors."""
    if u.dim() != 3 or u.shape != v.shape or u.dtype != v.dtype:
        raise ValueError("u, v must be [B, Ny, Nx] tensors of one dtype")
    b, ny, nx = u.shape
    g = Grid(nx, ny, lx, ly, b, F64 if u.dtype == torch.float64 else F32, layout)
    uo, vo = (torch.empty_like(u), torch.empty_like(v)) if out is None else out
    for name, t in (("u", u), ("v", v), ("u_out", uo), ("v_out", vo)):
        if not (t.is_cuda and t.dtype == u.dtype and t.is_contiguous()
                and tuple(t.shape) == (b, ny, nx)):
            raise ValueError("%s must be a contiguous %s cuda tensor of shape %s"
                             % (name, u.dtype, (b, ny, nx)))
    if coef is not None and not (coef.is_cuda and coef.dtype == torch.float32
                                 and coef.is_contiguous()
                                 and tuple(coef.shape) == (b, NCOEF, ny, nx)):
        raise ValueError("coef must be float32 [B, 64, Ny, Nx] contiguous on cuda")
    _check(_lib.ldsv_fv_step_noalloc(ctypes.byref(g), ctypes.byref(prm), _ptr(coef), _ptr(u),
                                     _ptr(v), _ptr(uo), _ptr(vo), nsteps, _stream()))
    return uo, vo


def adam_step(w, g, m, v, t, lr=1e-4, b1=0.9, b2=0.999, eps=1e-8):
    _check(_lib.ldsv_adam_step(_ptr(w), _ptr(g), _ptr(m), _ptr(v), w.numel(), t, lr, b1, b2, eps,
                               _stream()))


class FnoParams:
    """Device copy of one FNO (float32): lift_w [C, n_in], lift_b [C],
    spec_w [L, C_in, C_out, 2M, M, 2] (complex as re, im), point_w
    [L, C_out, C_in], point_b [L, C], proj_w [n_out, C], proj_b [n_out].
    The flux block's operators take n_in = 2 (u, v) and n_out = 4; the
    temporal correction n_in = 2 k_c and n_out = 2."""

    def __init__(self, lift_w, lift_b, spec, point_w, point_b, proj_w, proj_b):
        """spec: list over layers of complex [2M, M, C_in, C_out] tensors (the
        retained-row, k_x, in, out order), or of (re, im) pairs of real ones."""
        f32 = lambda t: torch.as_tensor(t).detach().to("cuda", torch.float32).contiguous()
        self.lift_w, self.lift_b = f32(lift_w), f32(lift_b)
        layers = []
        for R in spec:
            if isinstance(R, (tuple, list)):
                re, im = (torch.as_tensor(x, dtype=torch.float64) for x in R)
            else:
                R = torch.as_tensor(R)
                re, im = R.real.double(), R.imag.double()
            z = torch.stack([re, im], dim=-1)                 # [2M, M, Ci, Co, 2]
            layers.append(z.permute(2, 3, 0, 1, 4))           # [Ci, Co, 2M, M, 2]
        self.spec_w = f32(torch.stack(layers))
        self.point_w, self.point_b = f32(point_w), f32(point_b)
        self.proj_w, self.proj_b = f32(proj_w), f32(proj_b)
        L, C, _, two_m, M, _ = self.spec_w.shape
        self.n_in, self.n_out = self.lift_w.shape[1], self.proj_w.shape[0]
        self.c = Fno(C, L, M, self.n_in, self.n_out, self.lift_w.data_ptr(), self.lift_b.data_ptr(),
                     self.spec_w.data_ptr(), self.point_w.data_ptr(), self.point_b.data_ptr(),
                     self.proj_w.data_ptr(), self.proj_b.data_ptr())

    @classmethod
    def from_arrays(cls, a):
        """From the real arrays of synthetic_inputs.fno_weights."""
        import numpy as np
        return cls(a["P_w"], a["P_b"], [(l["R_re"], l["R_im"]) for l in a["layers"]],
                   np.stack([l["W"] for l in a["layers"]]),
                   np.stack([l["b"] for l in a["layers"]]), a["Q_w"], a["Q_b"])


class FluxNetParams:
    """The flux block's learnable parameters: uniform kernels stencil_w
    [2, 4, 20] (interpolation, derivative) and the two FNOs (either may be
    None)."""

    def __init__(self, stencil_w, fno_i=None, fno_d=None):
        self.stencil_w = torch.as_tensor(stencil_w).detach().to("cuda", torch.float32) \
            .reshape(2, 4, 20).contiguous()
        self.fno = [fno_i, fno_d]
        self.c = FluxNet()
        self.c.stencil_w = self.stencil_w.data_ptr()
        for g, f in enumerate(self.fno):
            self.c.fno[g] = ctypes.pointer(f.c) if f is not None else ctypes.POINTER(Fno)()


class FnoGradBuffers:
    """Zeroed float32 gradient buffers with the layouts of a FnoParams."""

    NAMES = ("lift_w", "lift_b", "spec_w", "point_w", "point_b", "proj_w", "proj_b")

    def __init__(self, fno):
        for k in self.NAMES:
            setattr(self, k, torch.zeros_like(getattr(fno, k)))
        self.c = FnoGrad(*[getattr(self, k).data_ptr() for k in self.NAMES])

    def tensors(self):
        return [getattr(self, k) for k in self.NAMES]

    def spec_complex(self):
        """spec_w as complex [L, 2M, M, C_in, C_out] (the oracle's R order)."""
        return torch.view_as_complex(self.spec_w.contiguous()).permute(0, 3, 4, 1, 2)


class FluxNetGradBuffers:
    """Gradients of a FluxNetParams (accumulated by the backward calls)."""

    def __init__(self, net):
        self.stencil_w = torch.zeros_like(net.stencil_w)
        self.fno = [FnoGradBuffers(f) if f is not None else None for f in net.fno]
        self.c = FluxNetGrad()
        self.c.stencil_w = self.stencil_w.data_ptr()
        for g, f in enumerate(self.fno):
            self.c.fno[g] = ctypes.pointer(f.c) if f is not None else ctypes.POINTER(FnoGrad)()

    def zero_(self):
        self.stencil_w.zero_()
        for f in self.fno:
            if f is not None:
                for t in f.tensors():
                    t.zero_()

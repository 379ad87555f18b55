"""Finite-volume residuals on a periodic 2D box (oracle, float64, torch CPU).

Grid (App. B.1, Fig. S1 staggered grid with periodic padding): the box
[0, Lx) x [0, Ly) has Nx x Ny cells, dx = Lx/Nx, cell (i, j) is centred at
((i+1/2)dx, (j+1/2)dy).  Arrays are [..., Ny, Nx] with x fastest (the paper's
T x n x n_y x n_x tensor layout, Sec. 4.1).  Periodic padding is a roll.

MAC layout (incompressible NS): u[j, i] lives on the west face of cell (i, j),
at (i dx, (j+1/2) dy); v[j, i] on the south face, at ((i+1/2) dx, j dy);
pressure at cell centres.

Collocated layout (Burgers): u and v both at cell centres.

Face stencils (App. B.2, Eq. S6 and S7; Sec. 3.4 Eqs. 5-7):
* derivative at the face between m and m+1 along an axis:
  (q[m-1] - 27 q[m] + 27 q[m+1] - q[m+2]) / (24 h)   (kernel S6);
* interpolation to that face: the paper calls it linear interpolation; the
  printed S7 row is a difference, which we read as the midpoint average
  (q[m] + q[m+1]) / 2;
* learned interpolation: a per-cell sum over a 16-point footprint of the 5x4
  window (4 points along the face normal, 5 across, minus the 4 corners).  Footprint point s = (a, b): along offset a in {-1,0,1,2}
  (index m+a), across offset b.  s = 0..11: a = s % 4 - 1, b = s // 4 - 1;
  s = 12: (0,-2), 13: (1,-2), 14: (0,2), 15: (1,2).  Kernels along y are the
  transpose of kernels along x.

Coefficient tensors are [B, 64, Ny, Nx]: channel 16*K + s for kind K:
  K0  u interpolated along x to the cell centre ((i+1/2)dx, (j+1/2)dy)
  K1  u interpolated along y to the corner (i dx, (j+1) dy)
  K2  v interpolated along x to the corner ((i+1) dx, j dy)
  K3  v interpolated along y to the cell centre
Each is the east (K0, K2) or north (K1, K3) face of the momentum control
volume of the owning index (i, j).  Flux differences therefore telescope and
the scheme conserves momentum whatever the coefficients are.

Flux block (Sec. 3.4, Eqs. 5-8): every face value is O_P + O_L + O_F.  Besides
the physics kernels above (O_P) and the per-cell coefficients, ``ns_rhs``
takes a ``flux`` record with the paper's spatially uniform learnable 5x4
kernels and the frequency-operator fields:
  wi [4, 20]  uniform learnable interpolation kernel per kind (O_L^(i))
  wd [4, 20]  uniform learnable derivative kernel per kind (O_L^(d)); the
              weights are dimensionless, the face derivative gets
              (1/h) sum_s wd[K, s] q_s with h the spacing along the normal
  fi [B, 4, Ny, Nx]  field added to the interpolated value of kind K at the
              face its cell owns (O_F^(i))
  fd [B, 4, Ny, Nx]  field added to the face derivative of kind K (O_F^(d))
The derivative kinds sit where the interpolation kinds do: K0 du/dx at the
cell centre, K1 du/dy at the corner, K2 dv/dx at the corner, K3 dv/dy at the
cell centre.  The uniform kernels cover the whole 5x4 window: footprint
points 0..15 as above, then the four corners 16: (-1,-2), 17: (2,-2),
18: (-1,2), 19: (2,2).  Any entry may be absent (None).  Each face value is
still single-valued, so the residual stays conservative.

Per-cell learned derivative stencils (the m = d operator in the per-cell
form, Sec. 3.4): ``dcoef`` [B, 64, Ny, Nx] holds dimensionless weights w on
the same 16-point footprint and kinds; the face derivative of kind K is
(1/h) sum_s w[16K + s] q_s with h the spacing along the face normal, in
place of the fourth-order kernel.  The learned module builds w from raw
network values so that it differentiates linear fields exactly.
"""
import math
import torch

# physics mask bits
ADVECTION = 1
VISCOSITY = 2
FORCING = 4
ALL_PHYSICS = 7

FOOTPRINT = [(s % 4 - 1, s // 4 - 1) for s in range(12)] + [(0, -2), (1, -2), (0, 2), (1, 2)]
NKIND = 4
NPOINT = 16
FOOTPRINT20 = FOOTPRINT + [(-1, -2), (2, -2), (-1, 2), (2, 2)]


def plain_deriv_coefficients(dtype=torch.float64):
    """The fourth-order derivative kernel (S6) as footprint weights, in units
    of 1/h: [1, -27, 27, -1]/24 at a = -1..2 on the row b = 0 (points 4..7)."""
    c = torch.zeros(NKIND * NPOINT, dtype=dtype)
    for k in range(NKIND):
        for s, w in zip(range(4, 8), (1.0, -27.0, 27.0, -1.0)):
            c[16 * k + s] = w / 24.0
    return c


def plain_coefficients(dtype=torch.float64):
    """The physics stencil c_P: weight 1/2 on the two points adjacent to the
    face (a = 0 and a = 1 at b = 0), zero elsewhere; the same for all 4 kinds."""
    c = torch.zeros(NKIND * NPOINT, dtype=dtype)
    for k in range(NKIND):
        c[16 * k + 5] = 0.5   # (a=0, b=0)
        c[16 * k + 6] = 0.5   # (a=1, b=0)
    return c


def sx(q, a):
    """q at x-index i+a (periodic)."""
    return torch.roll(q, shifts=-a, dims=-1)


def sy(q, b):
    """q at y-index j+b (periodic)."""
    return torch.roll(q, shifts=-b, dims=-2)


def _coef(c, kind, s):
    """Coefficient of footprint point s of kind K: either a scalar (uniform
    stencil given as a 64-vector) or a per-cell field [B, Ny, Nx]."""
    if c.dim() == 1:
        return c[16 * kind + s]
    return c[:, 16 * kind + s]


def interp_x(q, c, kind):
    """Face value between x-index i and i+1 at row j (owned by (i, j))."""
    out = 0.0
    for s, (a, b) in enumerate(FOOTPRINT):
        out = out + _coef(c, kind, s) * sx(sy(q, b), a)
    return out


def interp_y(q, c, kind):
    """Face value between y-index j and j+1 at column i (owned by (i, j))."""
    out = 0.0
    for s, (a, b) in enumerate(FOOTPRINT):
        out = out + _coef(c, kind, s) * sy(sx(q, b), a)
    return out


def deriv4_x(q, dx):
    """Fourth-order face derivative along x at the face between i and i+1 (S6)."""
    return (sx(q, -1) - 27.0 * q + 27.0 * sx(q, 1) - sx(q, 2)) / (24.0 * dx)


def deriv4_y(q, dy):
    return (sy(q, -1) - 27.0 * q + 27.0 * sy(q, 1) - sy(q, 2)) / (24.0 * dy)


def uniform_x(q, w):
    """Spatially uniform 5x4 kernel w [20] along x: sum_s w[s] q[j+b, i+a]."""
    out = 0.0
    for s, (a, b) in enumerate(FOOTPRINT20):
        out = out + w[s] * sx(sy(q, b), a)
    return out


def uniform_y(q, w):
    """The transpose kernel along y: sum_s w[s] q[j+a, i+b]."""
    out = 0.0
    for s, (a, b) in enumerate(FOOTPRINT20):
        out = out + w[s] * sy(sx(q, b), a)
    return out


def _flux_interp(q, flux, kind, along_x):
    """O_L^(i) + O_F^(i) part of the interpolated value of kind K (0 if absent)."""
    out = 0.0
    if flux is None:
        return out
    if flux.get("wi") is not None:
        w = flux["wi"][kind]
        out = out + (uniform_x(q, w) if along_x else uniform_y(q, w))
    if flux.get("fi") is not None:
        out = out + flux["fi"][:, kind]
    return out


def _flux_deriv(q, flux, kind, along_x, h):
    """O_L^(d) + O_F^(d) part of the face derivative of kind K (0 if absent)."""
    out = 0.0
    if flux is None:
        return out
    if flux.get("wd") is not None:
        w = flux["wd"][kind]
        out = out + (uniform_x(q, w) if along_x else uniform_y(q, w)) / h
    if flux.get("fd") is not None:
        out = out + flux["fd"][:, kind]
    return out


def _face_deriv(q, dcoef, kind, along_x, h):
    """Face derivative of kind K: the fourth-order kernel, or the per-cell
    learned weights dcoef (in units of 1/h) on the 16-point footprint."""
    if dcoef is None:
        return deriv4_x(q, h) if along_x else deriv4_y(q, h)
    return (interp_x(q, dcoef, kind) if along_x else interp_y(q, dcoef, kind)) / h


def ns_rhs(u, v, prm, coef=None, flux=None, dcoef=None):
    """Residual R(u) of the incompressible momentum equations without the
    pressure term, on the MAC grid (Eq. 4; App. B.2 S1-S5; App. C.1 S26).

    For the u control volume centred at (i dx, (j+1/2) dy) (App. B.2, S2, S3,
    S5):
      R_u = -(F_e - F_w)/dx - (G_n - G_s)/dy
            + nu [ (du/dx)_e - (du/dx)_w ]/dx + nu [ (du/dy)_n - (du/dy)_s ]/dy
            + f_x
    with advective fluxes F = (advecting u) * (advected u) on each face; the
    advecting velocity is the linear average of the normal velocity, the
    advected value comes from the interpolation stencil.  The v equation is
    the mirror image.  Forcing (App. C.1, forced flow): f = [A sin(k y) - d u,
    -d v] with y the u-point height, evaluated on the stage state.

    prm keys: dx, dy, nu, forcing_amp, forcing_k, drag, mask.
    coef: None for the physics stencil, else a 64-vector or [B, 64, Ny, Nx].
    flux: None, or the flux-block record (wi, wd, fi, fd) described above,
    whose terms add to the face values.
    dcoef: None for the fourth-order derivative, else per-cell derivative
    weights [B, 64, Ny, Nx] (dimensionless, see the module header).
    """
    dx, dy = prm["dx"], prm["dy"]
    mask = prm.get("mask", ALL_PHYSICS)
    c = plain_coefficients(u.dtype) if coef is None else coef
    ru = torch.zeros_like(u)
    rv = torch.zeros_like(v)
    if mask & ADVECTION:
        # u momentum: east face at the cell centre, north face at the corner
        ubar_c = 0.5 * (u + sx(u, 1))
        F = ubar_c * (interp_x(u, c, 0) + _flux_interp(u, flux, 0, True))
        vbar_n = 0.5 * (sx(sy(v, 1), -1) + sy(v, 1))     # v[j+1, i-1], v[j+1, i]
        G = vbar_n * (interp_y(u, c, 1) + _flux_interp(u, flux, 1, False))
        ru = ru - (F - sx(F, -1)) / dx - (G - sy(G, -1)) / dy
        # v momentum: east face at the corner, north face at the cell centre
        ubar_e = 0.5 * (sx(sy(u, -1), 1) + sx(u, 1))     # u[j-1, i+1], u[j, i+1]
        E = ubar_e * (interp_x(v, c, 2) + _flux_interp(v, flux, 2, True))
        vbar_c = 0.5 * (v + sy(v, 1))
        H = vbar_c * (interp_y(v, c, 3) + _flux_interp(v, flux, 3, False))
        rv = rv - (E - sx(E, -1)) / dx - (H - sy(H, -1)) / dy
    if mask & VISCOSITY:
        nu = prm["nu"]
        ux = _face_deriv(u, dcoef, 0, True, dx) + _flux_deriv(u, flux, 0, True, dx)
        uy = _face_deriv(u, dcoef, 1, False, dy) + _flux_deriv(u, flux, 1, False, dy)
        vx = _face_deriv(v, dcoef, 2, True, dx) + _flux_deriv(v, flux, 2, True, dx)
        vy = _face_deriv(v, dcoef, 3, False, dy) + _flux_deriv(v, flux, 3, False, dy)
        ru = ru + nu * ((ux - sx(ux, -1)) / dx + (uy - sy(uy, -1)) / dy)
        rv = rv + nu * ((vx - sx(vx, -1)) / dx + (vy - sy(vy, -1)) / dy)
    if mask & FORCING:
        ny = u.shape[-2]
        y = (torch.arange(ny, dtype=u.dtype) + 0.5) * dy
        fx = prm.get("forcing_amp", 0.0) * torch.sin(prm.get("forcing_k", 0.0) * y)
        drag = prm.get("drag", 0.0)
        ru = ru + fx.view(-1, 1) - drag * u
        rv = rv - drag * v
    return ru, rv


def upwind2_x(q, a):
    """Second-order linear-upwind value at the face between i and i+1,
    biased by the sign of the face velocity a (our reading: a > 0 takes the
    left-biased value (-q[i-1] + 3 q[i])/2, else (3 q[i+1] - q[i+2])/2)."""
    left = -0.5 * sx(q, -1) + 1.5 * q
    right = 1.5 * sx(q, 1) - 0.5 * sx(q, 2)
    return torch.where(a > 0, left, right)


def upwind2_y(q, b):
    low = -0.5 * sy(q, -1) + 1.5 * q
    high = 1.5 * sy(q, 1) - 0.5 * sy(q, 2)
    return torch.where(b > 0, low, high)


def burgers_rhs(u, v, prm):
    """Residual of 2D viscous Burgers, du/dt = nu lap u - u . grad u (App. C.1
    S25), on the collocated grid (our reading: flux form minus q div, which
    equals the advective form of S25 and the conservative form of Eq. 1 when
    the field is solenoidal).

    For each component q in {u, v}, with face-normal velocities a (east) and
    b (north) as central averages and q~ by linear upwind:
      R_q = -[(a_e q~_e - a_w q~_w)/dx + (b_n q~_n - b_s q~_s)/dy]
            + q [(a_e - a_w)/dx + (b_n - b_s)/dy]
            + nu [(q[i+1] - 2q + q[i-1])/dx^2 + (q[j+1] - 2q + q[j-1])/dy^2]
    The viscous term is the compact second-order face-derivative difference.
    """
    dx, dy = prm["dx"], prm["dy"]
    mask = prm.get("mask", ALL_PHYSICS)
    a = 0.5 * (u + sx(u, 1))
    b = 0.5 * (v + sy(v, 1))
    out = []
    for q in (u, v):
        r = torch.zeros_like(q)
        if mask & ADVECTION:
            fe = a * upwind2_x(q, a)
            fn = b * upwind2_y(q, b)
            flux_div = (fe - sx(fe, -1)) / dx + (fn - sy(fn, -1)) / dy
            vel_div = (a - sx(a, -1)) / dx + (b - sy(b, -1)) / dy
            r = r - flux_div + q * vel_div
        if mask & VISCOSITY:
            nu = prm["nu"]
            r = r + nu * ((sx(q, 1) - 2.0 * q + sx(q, -1)) / dx ** 2
                          + (sy(q, 1) - 2.0 * q + sy(q, -1)) / dy ** 2)
        out.append(r)
    return out[0], out[1]


def grid_params(nx, ny, lx=2 * math.pi, ly=2 * math.pi, **kw):
    prm = {"nx": nx, "ny": ny, "lx": lx, "ly": ly, "dx": lx / nx, "dy": ly / ny,
           "nu": 0.0, "forcing_amp": 0.0, "forcing_k": 0.0, "drag": 0.0,
           "mask": ALL_PHYSICS, "dt": 0.0}
    prm.update(kw)
    return prm

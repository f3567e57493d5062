"""Seeded synthetic workloads shared by the oracle tests, the GPU tests and the benchmark.

This module only draws random numbers and lays out grids.  It holds none of the
method's arithmetic (no residual, no derivative, no Krylov or Newton step), so
the CPU oracle and the HIP path can both take their inputs from here without
sharing any code that computes the method.

Every generator takes an explicit seed and uses ``numpy.random.default_rng``.
State vectors are flat float64 arrays in the layout both sides use:

* 1D Burgers: ``u[i]``, ``i = 0..nx-1``.
* 2D two-field problems (Burgers, Gray-Scott): two planes, each row-major,
  ``x[f*nx*ny + j*nx + i]`` for field ``f``, row ``j`` (y), column ``i`` (x).
* Helmholtz-Kerr: complex field, real and imaginary parts interleaved,
  ``x[2*(j*nx + i) + c]`` with ``c = 0`` (real) or ``1`` (imaginary).

The parameter sets follow the paper's benchmark problems (its Section 3.2 and
Appendix A) where the paper fixes them, and the workload definitions of this
project otherwise; every choice the paper leaves open is listed with its
reading in the design notes.
"""

from __future__ import annotations

import math

import numpy as np

# ---------------------------------------------------------------------------
# Problem specifications (plain numbers; both sides build their own objects)
# ---------------------------------------------------------------------------


def burgers1d_spec(nx: int = 256, nu: float = 0.01, dt: float = 1e-3, theta: float = 1.0) -> dict:
    """1D viscous Burgers on [0,1) periodic, h = 1/nx (backward Euler by default)."""
    return dict(kind="burgers1d", nx=nx, ny=1, hx=1.0 / nx, hy=1.0, dt=dt, theta=theta, nu=nu)


def burgers2d_spec(n: int = 2048, nu: float = 1e-3, dt: float = 5e-4, theta: float = 0.5) -> dict:
    """2D viscous Burgers on [0,2pi)^2 periodic (Crank-Nicolson by default, Appendix A.1)."""
    h = 2.0 * math.pi / n
    return dict(kind="burgers2d", nx=n, ny=n, hx=h, hy=h, dt=dt, theta=theta, nu=nu)


def grayscott_spec(n: int = 1024, D: float = 2e-5, Dv: float = 1e-5, F: float = 0.04, k: float = 0.06,
                   dt: float = 1.0, theta: float = 1.0, h: float | None = None) -> dict:
    """Gray-Scott two-species reaction-diffusion, periodic.

    The grid spacing defaults to h = sqrt(D*dt), i.e. a diffusion Courant number
    of one in the paper's reaction-diffusion rule dt = C h^2 / D with C = 1.
    """
    if h is None:
        h = math.sqrt(D * dt)
    return dict(kind="grayscott", nx=n, ny=n, hx=h, hy=h, dt=dt, theta=theta, D=D, Dv=Dv, F=F, k=k)


def kerr_spec(n: int = 1024, chi3: float = 0.1, eps_re: float = 1.0, eps_im: float = 0.0,
              cells_per_wavelength: float = 64.0) -> dict:
    """Scalar Helmholtz-Kerr on an n x n node grid, PEC boundary nodes, h = 1 (grid units)."""
    return dict(kind="kerr", nx=n, ny=n, hx=1.0, hy=1.0, dt=0.0, theta=1.0,
                k0=2.0 * math.pi / cells_per_wavelength, eps_re=eps_re, eps_im=eps_im, chi3=chi3)


def rd2d_spec(n: int = 512, D: float = 0.01, C: float = 1.0, theta: float = 0.5, ny: int | None = None) -> dict:
    """Scalar reaction-diffusion u_t = D Lap u - u^3 on the node grid of [0,1]^2.

    Homogeneous Dirichlet boundary nodes, Crank-Nicolson, and the paper's
    reaction-diffusion step rule dt = C h^2 / D (C = 1 by default).
    """
    ny = n if ny is None else ny
    hx = 1.0 / (n - 1)
    hy = 1.0 / (ny - 1)
    return dict(kind="rd2d", nx=n, ny=ny, hx=hx, hy=hy, dt=C * hx * hx / D, theta=theta, D=D)


def suolson_spec(n: int = 512, xi: float = 0.1, C: float = 1.0, theta: float = 0.5, L: float = 10.0,
                 ny: int | None = None, periodic_y: bool = False) -> dict:
    """Su-Olson radiation diffusion on the node grid of [-L/2, L/2]^2 (Appendix A.2): Dirichlet
    boundary nodes, Crank-Nicolson, dt = min(C h^2 / D, C / xi) with D = 1/3.  With
    ``periodic_y`` (the classic 1D-profile configuration) the ny rows are periodic nodes of
    [-L/2, L/2) (hy = L / ny) and only the first and last columns are Dirichlet nodes."""
    ny = n if ny is None else ny
    hx = L / (n - 1)
    hy = L / ny if periodic_y else L / (ny - 1)
    dt = min(C * min(hx, hy) ** 2 / (1.0 / 3.0), C / xi)
    spec = dict(kind="suolson", nx=n, ny=ny, hx=hx, hy=hy, dt=dt, theta=theta, xi=xi)
    if periodic_y:
        spec["periodic_y"] = True
    return spec


def suolson_box_initial(n: int = 512, ny: int | None = None, L: float = 10.0, Q0: float = 1.0,
                        x0: float = 0.5) -> tuple[np.ndarray, np.ndarray]:
    """(x^0, source) of the classic 1D-profile Su-Olson configuration: cold start (U = V = 0)
    and the central stationary box source Q0 on |x| <= x0 (every row; the classic problem's
    half-width x0 = 1/2), zero on the boundary columns."""
    ny = n if ny is None else ny
    x = np.linspace(-L / 2, L / 2, n)
    q = np.where(np.abs(x) <= x0 + 1e-12, Q0, 0.0)
    q[0] = q[-1] = 0.0
    Q = np.tile(q, (ny, 1))
    return np.zeros(2 * n * ny), np.concatenate([Q.ravel(), np.zeros(n * ny)])


def suolson_initial(n: int = 512, seed: int = 0, ny: int | None = None, L: float = 10.0, Q0: float = 1.0,
                    sigma: float = 0.4, R: float = 2.0) -> tuple[np.ndarray, np.ndarray]:
    """(x^0, source) of the dynamic Su-Olson configuration: decaying concentric rings in U (radii
    1, 2, 3, amplitudes 1, 1/2, 1/4, width 0.2) with V = U / 2, and the Gaussian source of
    amplitude Q0 and width sigma at a seeded angle on the orbit of radius R; zero on the boundary."""
    ny = n if ny is None else ny
    x = np.linspace(-L / 2, L / 2, n)[None, :]
    y = np.linspace(-L / 2, L / 2, ny)[:, None]
    r = np.sqrt(x * x + y * y)
    U = sum(a * np.exp(-((r - rk) ** 2) / (2 * 0.2 ** 2)) for rk, a in ((1.0, 1.0), (2.0, 0.5), (3.0, 0.25)))
    ang = np.random.default_rng(seed).uniform(0.0, 2.0 * np.pi)
    Q = Q0 * np.exp(-((x - R * np.cos(ang)) ** 2 + (y - R * np.sin(ang)) ** 2) / (2 * sigma ** 2)) * np.ones((ny, n))
    V = 0.5 * U
    for F in (U, V, Q):
        F[0, :] = F[-1, :] = 0.0
        F[:, 0] = F[:, -1] = 0.0
    return np.concatenate([U.ravel(), V.ravel()]), np.concatenate([Q.ravel(), np.zeros(n * ny)])


def maxwell_spec(n: int = 512, omega: float = 2.5, chi: float = 0.05, loss: float = 0.05,
                 ny: int | None = None) -> dict:
    """Paper-form Maxwell-Kerr (2D TE, Appendix A.4) on the node grid of [0,1]^2 with PEC
    boundary nodes; mu0 = eps0 = 1, so the frequency omega is stored as k0."""
    ny = n if ny is None else ny
    return dict(kind="maxwell", nx=n, ny=ny, hx=1.0 / (n - 1), hy=1.0 / (ny - 1), dt=0.0, theta=1.0,
                k0=omega, eps_im=loss, chi3=chi)


def maxwell_source(n: int = 512, omega: float = 2.5, kind: str = "dipole", sigma: float = 0.05,
                   x0: float = 0.5, ys: tuple = (0.4, 0.6), ny: int | None = None) -> np.ndarray:
    """f = i omega J for the paper's two currents (J_y = 0): a Gaussian J_x at (x0, ys[0]) or the
    antisymmetric dipole (Gaussians at (x0, ys[0]) minus (x0, ys[1])); zero on the boundary nodes.
    Planes (Re fx, Im fx, Re fy, Im fy)."""
    ny = n if ny is None else ny
    x = np.linspace(0.0, 1.0, n)[None, :]
    y = np.linspace(0.0, 1.0, ny)[:, None]

    def g(yc):
        return np.exp(-((x - x0) ** 2 + (y - yc) ** 2) / (2 * sigma * sigma))

    J = g(ys[0]) if kind == "gaussian" else g(ys[0]) - g(ys[1])
    J = J * np.ones((ny, n))
    J[0, :] = J[-1, :] = 0.0
    J[:, 0] = J[:, -1] = 0.0
    z = np.zeros(n * ny)
    return np.concatenate([z, (omega * J).ravel(), z, z])


def n_unknowns(spec: dict) -> int:
    """Number of real unknowns of a problem spec."""
    cells = spec["nx"] * spec["ny"]
    if spec["kind"] == "maxwell":
        return 4 * cells
    return cells if spec["kind"] in ("burgers1d", "rd2d") else 2 * cells


# ---------------------------------------------------------------------------
# Initial data and sources
# ---------------------------------------------------------------------------


def burgers1d_initial(nx: int = 256, seed: int = 0, noise: float = 1e-3) -> np.ndarray:
    """u0 = sin(2 pi x_i) + noise * N(0,1), x_i = i/nx."""
    rng = np.random.default_rng(seed)
    x = np.arange(nx, dtype=np.float64) / nx
    return np.sin(2.0 * np.pi * x) + noise * rng.standard_normal(nx)


def grayscott_initial(n: int = 1024, seed: int = 0, patches: int = 16, side_frac: float = 1.0 / 32,
                      noise: float = 0.01, ny: int | None = None) -> np.ndarray:
    """Background (u, v) = (0, 1) with square patches (0.25, 0.5) plus Gaussian noise.

    ``patches`` squares of side ``max(1, round(n*side_frac))`` cells are placed
    at seeded positions (periodic wrap); both fields then get ``noise*N(0,1)``.
    """
    ny = n if ny is None else ny
    nx = n
    rng = np.random.default_rng(seed)
    u = np.zeros((ny, nx))
    v = np.ones((ny, nx))
    side = max(1, int(round(min(nx, ny) * side_frac)))
    for _ in range(patches):
        j0 = int(rng.integers(0, ny))
        i0 = int(rng.integers(0, nx))
        rows = (j0 + np.arange(side)) % ny
        cols = (i0 + np.arange(side)) % nx
        u[np.ix_(rows, cols)] = 0.25
        v[np.ix_(rows, cols)] = 0.5
    u += noise * rng.standard_normal((ny, nx))
    v += noise * rng.standard_normal((ny, nx))
    return np.concatenate([u.ravel(), v.ravel()])


def burgers2d_initial(n: int = 2048, seed: int = 0, modes: int = 32, kmax: int = 8,
                      energy: float = 0.5) -> np.ndarray:
    """Random-Fourier velocity field on [0,2pi)^2 with mean kinetic energy ``energy``.

    Each component is a sum of ``modes`` waves a_m cos(k_m . x + phi_m) with
    integer wavevectors k_m drawn from {-kmax..kmax}^2 without the origin,
    a_m ~ N(0,1)/|k_m| and phi_m ~ U[0, 2pi).  The pair is then scaled so that
    0.5 * mean(u^2 + v^2) equals ``energy``.
    """
    rng = np.random.default_rng(seed)
    h = 2.0 * np.pi / n
    coord = np.arange(n) * h
    comps = []
    for _ in range(2):
        # cos(kx x + ky y + phi) = cos(kx x + phi) cos(ky y) - sin(kx x + phi) sin(ky y):
        # the field is a rank-2*modes product (rows y, columns x)
        A = np.empty((n, 2 * modes))
        B = np.empty((2 * modes, n))
        for m in range(modes):
            while True:
                kx, ky = (int(t) for t in rng.integers(-kmax, kmax + 1, size=2))
                if kx != 0 or ky != 0:
                    break
            amp = rng.standard_normal() / math.hypot(kx, ky)
            phi = rng.uniform(0.0, 2.0 * np.pi)
            A[:, 2 * m] = np.cos(ky * coord)
            A[:, 2 * m + 1] = -np.sin(ky * coord)
            B[2 * m] = amp * np.cos(kx * coord + phi)
            B[2 * m + 1] = amp * np.sin(kx * coord + phi)
        comps.append(A @ B)
    u, v = comps
    ke = 0.5 * np.mean(u * u + v * v)
    s = math.sqrt(energy / ke)
    return np.concatenate([(s * u).ravel(), (s * v).ravel()])


def taylor_green(n: int) -> np.ndarray:
    """Taylor-Green vortex u = sin x cos y, v = -cos x sin y on [0,2pi)^2 (Appendix A.1)."""
    h = 2.0 * np.pi / n
    c = np.arange(n) * h
    X = c[None, :]
    Y = c[:, None]
    u = np.sin(X) * np.cos(Y)
    v = -np.cos(X) * np.sin(Y)
    return np.concatenate([u.ravel(), v.ravel()])


def double_shear_layer(n: int, rho: float = 30.0, delta: float = 0.05) -> np.ndarray:
    """Double shear layer on [0,2pi)^2 (Appendix A.1): u = tanh(rho (y - pi/2)) for y <= pi,
    tanh(rho (3 pi/2 - y)) above; v = delta sin x."""
    h = 2.0 * np.pi / n
    c = np.arange(n) * h
    X = c[None, :]
    Y = c[:, None]
    u = np.where(Y <= np.pi, np.tanh(rho * (Y - np.pi / 2)), np.tanh(rho * (1.5 * np.pi - Y))) * np.ones_like(X)
    v = delta * np.sin(X) * np.ones_like(Y)
    return np.concatenate([u.ravel(), v.ravel()])


def burgers2d_cfl_dt(x: np.ndarray, n: int, nu: float, C: float = 1.0) -> float:
    """The paper's Burgers step rule (Appendix A.1) on the state x of an n x n grid of [0,2pi)^2:
    dt = C min(h / max|u|, h / max|v|, 1 / (2 nu (2 / h^2)))."""
    h = 2.0 * np.pi / n
    u = np.abs(x[: n * n]).max()
    v = np.abs(x[n * n:]).max()
    cands = [1.0 / (2.0 * nu * (2.0 / (h * h)))]
    if u > 0:
        cands.append(h / u)
    if v > 0:
        cands.append(h / v)
    return C * min(cands)


def burgers2d_paper_case(name: str, n: int = 256, nu: float = 0.05, C: float = 1.0) -> tuple[dict, np.ndarray]:
    """(spec, U^0) of the paper's periodic Burgers set-ups: ``tgv`` (Taylor-Green vortex) or
    ``dsl`` (double shear layer), Crank-Nicolson, nu = 0.05 (the paper's TGV figure), the time
    step from the CFL rule on the initial state."""
    x0 = taylor_green(n) if name == "tgv" else double_shear_layer(n)
    spec = burgers2d_spec(n, nu=nu, dt=burgers2d_cfl_dt(x0, n, nu, C), theta=0.5)
    return spec, x0


def kerr_gaussian_source(n: int = 1024, amp: float = 0.1, sigma: float = 4.0,
                         center: tuple[float, float] | None = None, ny: int | None = None) -> np.ndarray:
    """Real Gaussian source f on the node grid, zero on the PEC boundary, interleaved complex."""
    ny = n if ny is None else ny
    nx = n
    cx = (nx - 1) / 2.0 if center is None else center[0]
    cy = (ny - 1) / 2.0 if center is None else center[1]
    i = np.arange(nx)[None, :]
    j = np.arange(ny)[:, None]
    g = amp * np.exp(-((i - cx) ** 2 + (j - cy) ** 2) / (2.0 * sigma * sigma))
    g[0, :] = 0.0
    g[-1, :] = 0.0
    g[:, 0] = 0.0
    g[:, -1] = 0.0
    out = np.zeros((ny, nx, 2))
    out[..., 0] = g
    return out.ravel()


def rd2d_initial(n: int = 512, seed: int = 0, profile: str = "multigauss", ny: int | None = None,
                 k: int = 4) -> np.ndarray:
    """Initial concentration of the reaction-diffusion problem, zero on the boundary nodes.

    Profiles (the paper's three, Appendix A.3): ``gaussian`` (one peak at the
    centre, sigma 0.1), ``multigauss`` (four peaks at seeded positions in
    [0.2, 0.8]^2 with seeded widths in [0.05, 0.1]), ``sine``
    (|sin(k pi x) sin(k pi y)|).  Unit amplitude.
    """
    ny = n if ny is None else ny
    x = np.linspace(0.0, 1.0, n)[None, :]
    y = np.linspace(0.0, 1.0, ny)[:, None]
    if profile == "gaussian":
        u = np.exp(-((x - 0.5) ** 2 + (y - 0.5) ** 2) / (2 * 0.1 ** 2))
    elif profile == "multigauss":
        rng = np.random.default_rng(seed)
        cx, cy = rng.uniform(0.2, 0.8, 4), rng.uniform(0.2, 0.8, 4)
        sig = rng.uniform(0.05, 0.1, 4)
        u = sum(np.exp(-((x - cx[q]) ** 2 + (y - cy[q]) ** 2) / (2 * sig[q] ** 2)) for q in range(4))
    elif profile == "sine":
        u = np.abs(np.sin(k * np.pi * x) * np.sin(k * np.pi * y))
    else:
        raise KeyError(profile)
    u = np.array(u, dtype=np.float64) * np.ones((ny, n))
    u[0, :] = 0.0
    u[-1, :] = 0.0
    u[:, 0] = 0.0
    u[:, -1] = 0.0
    return u.ravel()


def random_vector(n: int, seed: int, scale: float = 1.0) -> np.ndarray:
    """A seeded N(0, scale^2) vector (Krylov directions and generic test data)."""
    return scale * np.random.default_rng(seed).standard_normal(n)


# ---------------------------------------------------------------------------
# Named configurations
# ---------------------------------------------------------------------------


def config(name: str, seed: int = 0, n: int | None = None) -> tuple[dict, np.ndarray, np.ndarray | None]:
    """Return (spec, x_prev, source) for a named workload, optionally at another size.

    Names: ``burgers1d`` (N=256 by default), ``grayscott`` (1024^2),
    ``burgers2d`` (2048^2), ``kerr`` (1024^2, chi3 = 0.1), ``rd2d`` (512^2,
    the paper's GPU reaction-diffusion grid, multi-Gaussian start), ``suolson``
    (512^2, rings and orbiting source), ``suolson1d`` (512^2, periodic rows,
    cold start with the central box source), ``maxwell`` (512^2, dipole).
    """
    if name == "burgers1d":
        nx = 256 if n is None else n
        spec = burgers1d_spec(nx)
        return spec, burgers1d_initial(nx, seed), None
    if name == "grayscott":
        nn = 1024 if n is None else n
        spec = grayscott_spec(nn)
        return spec, grayscott_initial(nn, seed), None
    if name == "burgers2d":
        nn = 2048 if n is None else n
        spec = burgers2d_spec(nn)
        return spec, burgers2d_initial(nn, seed), None
    if name == "kerr":
        nn = 1024 if n is None else n
        spec = kerr_spec(nn)
        return spec, np.zeros(2 * nn * nn), kerr_gaussian_source(nn)
    if name == "rd2d":
        nn = 512 if n is None else n
        spec = rd2d_spec(nn)
        return spec, rd2d_initial(nn, seed), None
    if name == "maxwell":
        nn = 512 if n is None else n
        return maxwell_spec(nn), np.zeros(4 * nn * nn), maxwell_source(nn)
    if name == "suolson":
        nn = 512 if n is None else n
        x0, src = suolson_initial(nn, seed)
        return suolson_spec(nn), x0, src
    if name == "suolson1d":
        nn = 512 if n is None else n
        x0, src = suolson_box_initial(nn)
        return suolson_spec(nn, periodic_y=True), x0, src
    raise KeyError(name)


def serving_stream(count: int = 2000, seed: int = 0, rate: float = 1.0) -> list[dict]:
    """Poisson stream of implicit-step requests mixing 1D Burgers and 2D Gray-Scott.

    Each request: type Bernoulli(1/2); 1D Burgers N = 2^e, e ~ U{8..16}, with
    dt(N) = 1e-3 (256/N)^2 (keeping the N=256 diffusion number); Gray-Scott side
    2^e, e ~ U{6..10}.  Arrival gaps are exponential with mean 1/rate seconds.
    Initial data come from the per-request seed.
    """
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for r in range(count):
        t += float(rng.exponential(1.0 / rate))
        kind = "burgers1d" if rng.random() < 0.5 else "grayscott"
        if kind == "burgers1d":
            e = int(rng.integers(8, 17))
            size = 2 ** e
        else:
            e = int(rng.integers(6, 11))
            size = 2 ** e
        out.append(dict(id=r, arrival=t, kind=kind, size=size, seed=int(rng.integers(0, 2**31 - 1))))
    return out


def serving_request_inputs(req: dict) -> tuple[dict, np.ndarray]:
    """(spec, x_prev) of one serving request."""
    if req["kind"] == "burgers1d":
        nx = req["size"]
        spec = burgers1d_spec(nx, dt=1e-3 * (256.0 / nx) ** 2)
        return spec, burgers1d_initial(nx, req["seed"])
    n = req["size"]
    spec = grayscott_spec(n)
    return spec, grayscott_initial(n, req["seed"])

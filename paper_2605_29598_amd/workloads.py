"""Seeded synthetic workloads: mesh/physics/solver settings and initial states.

This module holds no arithmetic of the DG method: it only describes the test
problems (domains, stratified backgrounds, perturbations, noise) and turns
primitive fields given at node coordinates into conserved variables. Both
the HIP path and its CPU checker take their inputs from here.

Backgrounds follow Sec. 4: the isothermal hydrostatic state of the inertia-
gravity-wave test (p = p_s exp(-delta z), delta = g / (R T0)) and the
constant-N stratification in Exner form of the orography tests. Reference
surface pressure p_s = 1e5 Pa where the paper leaves it open.
"""
import math
from dataclasses import dataclass, field, asdict
import numpy as np

GAMMA, RGAS, GRAV = 1.4, 287.0, 9.81
CP = GAMMA * RGAS / (GAMMA - 1.0)
P_REF = 1.0e5

FLAT, BELL, GAUSS = 0, 1, 2
R1, R2 = 1, 2


@dataclass
class MeshSpec:
    Lx: float
    Ly: float
    Lz: float
    nx: int
    ny: int
    nz: int
    degree: int
    periodic_x: int = 1
    periodic_y: int = 1
    terrain: int = FLAT
    h0: float = 0.0
    a: float = 1.0
    xc: float = 0.0
    yc: float = 0.0
    ref_boxes: list = field(default_factory=list)


@dataclass
class PhysSpec:
    gamma: float = GAMMA
    R: float = RGAS
    g: float = GRAV
    f: float = 0.0
    sponge_zB: float = 0.0
    sponge_zT: float = 1.0
    sponge_lam: float = 0.0
    sponge_u: tuple = (0.0, 0.0, 0.0)
    sponge_xw: float = 0.0   # widths of the lateral sponge layers at both ends of x and y (0 = none)
    sponge_yw: float = 0.0
    slice: int = 0           # vertical-slice equations (one periodic element in y)


@dataclass
class NumSpec:
    dt: float = 1.0
    scheme: int = R2
    picard_tol: float = 1e-10
    picard_max: int = 20
    gmres_tol: float = 1e-10
    gmres_restart: int = 30
    gmres_max: int = 500
    fixed_iterations: bool = False


@dataclass
class Workload:
    name: str
    mesh: MeshSpec
    phys: PhysSpec
    num: NumSpec
    steps: int
    background: str          # "isothermal" or "stratified"
    T0: float                # isothermal temperature or surface potential temperature
    N: float = 0.0
    U: float = 0.0
    pert: str = "none"       # "gauss" (radius a_p), "igw" (sin(pi z/H)/(1+(x-xc)^2/a_p^2)) or "bretherton"
    pert_amp: float = 0.0
    pert_a: float = 1.0
    pert_xc: float = 0.0
    pert_yc: float = 0.0
    pert_zc: float = 0.0
    noise: float = 0.0
    seed: int = 0

    def as_dict(self):
        return asdict(self)


# --------------------------------------------------------------- workloads
def tiny_box(degree=2, scheme=R2):
    """10x10x10 km box, 4x4x4 elements, isothermal 250 K rest state, f = 1e-4,
    Gaussian theta' 0.01 K of radius 2 km at the centre, 1e-6 noise, dt = 2 s."""
    return Workload(
        name="tiny_box_4x4x4_r%d" % degree,
        mesh=MeshSpec(10e3, 10e3, 10e3, 4, 4, 4, degree),
        phys=PhysSpec(f=1e-4),
        num=NumSpec(dt=2.0, scheme=scheme, gmres_tol=1e-10),
        steps=10, background="isothermal", T0=250.0,
        pert="gauss", pert_amp=0.01, pert_a=2e3, pert_xc=5e3, pert_yc=5e3, pert_zc=5e3,
        noise=1e-6, seed=0)


def igw_channel(nx=120, ny=40, nz=10, degree=3, scheme=R2):
    """Rotating inertia-gravity-wave channel 3000x1000x10 km: N = 0.01, theta0 =
    300 K, U = 20 m/s, f = 1e-4, theta' = 0.01 sin(pi z/H)/(1+(x-xc)^2/a^2),
    a = 100 km, xc = 1500 km; dt = 20 s, 200 steps."""
    return Workload(
        name="igw_channel_%dx%dx%d_r%d" % (nx, ny, nz, degree),
        mesh=MeshSpec(3000e3, 1000e3, 10e3, nx, ny, nz, degree),
        phys=PhysSpec(f=1e-4),
        num=NumSpec(dt=20.0, scheme=scheme),
        steps=200, background="stratified", T0=300.0, N=0.01, U=20.0,
        pert="igw", pert_amp=0.01, pert_a=100e3, pert_xc=1500e3, seed=1)


def orography(nx=64, ny=64, nz=24, degree=4, scheme=R2, refined=False):
    """Stratified rotating flow over a Gaussian hill (h0 = 400 m, half-width
    2 km, centre (30, 30) km) in a 60x60x20 km Gal-Chen box: theta_ref =
    293.15 K, N = 0.01, U = 10 m/s, f = 1e-4, Rayleigh sponge above 12 km with
    lambda*dt = 1.2; dt = 4 s, 500 steps. `refined` gives the non-conforming
    variant: two nested 2:1 levels around the hill."""
    dt = 4.0
    boxes = []
    if refined:
        boxes = [(25e3, 35e3, 25e3, 35e3, 0.0, 6e3), (27.5e3, 32.5e3, 27.5e3, 32.5e3, 0.0, 3e3)]
    return Workload(
        name="orography_%dx%dx%d_r%d%s" % (nx, ny, nz, degree, "_amr" if refined else ""),
        mesh=MeshSpec(60e3, 60e3, 20e3, nx, ny, nz, degree, terrain=GAUSS, h0=400.0,
                      a=2e3, xc=30e3, yc=30e3, ref_boxes=boxes),
        phys=PhysSpec(f=1e-4, sponge_zB=12e3, sponge_zT=20e3, sponge_lam=1.2 / dt,
                      sponge_u=(10.0, 0.0, 0.0)),
        num=NumSpec(dt=dt, scheme=scheme),
        steps=500, background="stratified", T0=293.15, N=0.01, U=10.0,
        seed=3 if not refined else 4)


def advected_bubble(nx=8, ny=4, nz=4, degree=3, scheme=R2, amp=10.0):
    """A warm bubble carried by a uniform wind through a periodic 40 x 20 x 10
    km box (stratified rest state N = 0.01, theta0 = 300 K, f = 1e-4,
    U = 20 m/s along x; Gaussian theta' of `amp` K and radius 2 km at
    (8, 10, 4) km), dt = 2 s: the feature that a moving refinement box
    follows in the adaptive runs."""
    return Workload(
        name="advected_bubble_%dx%dx%d_r%d" % (nx, ny, nz, degree),
        mesh=MeshSpec(40e3, 20e3, 10e3, nx, ny, nz, degree),
        phys=PhysSpec(f=1e-4),
        num=NumSpec(dt=2.0, scheme=scheme),
        steps=200, background="stratified", T0=300.0, N=0.01, U=20.0,
        pert="gauss", pert_amp=amp, pert_a=2e3, pert_xc=8e3, pert_yc=10e3, pert_zc=4e3, seed=11)


def hill_benchmark(rotating=True, nx=30, ny=20, nz=8, degree=4, scheme=R2, nonconforming=False):
    """Benchmark flow over orography of Sec. 4.3: a 60 x 40 x 16 km Gal-Chen box
    over the bell mountain h0 / (1 + r^2/a^2) (h0 = 400 m, a = 1 km, centre
    (30, 20) km), periodic in x and y; stratified rest-frame background
    theta_ref = 293.15 K, N = 0.01, uniform wind U = 10 m/s along x; Rayleigh
    damping in the first and last 20 km of x, the first and last 10 km of y
    and the top 6 km, lambda*dt = 1.2; 30 x 20 x 8 elements at r = 4
    (500 m effective resolution), dt = 8 s, 8 h; f = 1e-4 (rotating run) or 0.
    With periodic y the geostrophic pressure correction of the rotating run
    cannot be represented and is left out, as for the orography box.

    Non-conforming variant (the second pair of runs of the section): base
    elements of 4 km (1 km effective resolution at r = 4: 15 x 10 x 4), one
    level of refinement where x in [20, 40] km, y in [10, 30] km and z <= 7 km,
    a second where z <= 2 km, down to 1 km elements (250 m effective). The
    second box is drawn one level-1 element inside the first in x and y so that
    the mesh is 2:1 balanced as built (the section's mesh library balances by
    itself, which is not specified): 1,468 elements and 183,500 nodes per
    field, against the section's 1,594 and 199,250. dt = 4 s: at 8 s the
    advective Courant number on the 1 km elements (about 0.1) exceeds the
    explicit tableau's limit."""
    dt = 4.0 if nonconforming else 8.0
    boxes = []
    if nonconforming:
        nx, ny, nz = 15, 10, 4
        boxes = [(20e3, 40e3, 10e3, 30e3, 0.0, 7e3), (22e3, 38e3, 12e3, 28e3, 0.0, 2e3)]
    return Workload(
        name="hill_benchmark%s%s_%dx%dx%d_r%d" % ("_nc" if nonconforming else "", "_rotating" if rotating else "",
                                                  nx, ny, nz, degree),
        mesh=MeshSpec(60e3, 40e3, 16e3, nx, ny, nz, degree, terrain=BELL, h0=400.0, a=1e3, xc=30e3, yc=20e3,
                      ref_boxes=boxes),
        phys=PhysSpec(f=1e-4 if rotating else 0.0, sponge_zB=10e3, sponge_zT=16e3, sponge_lam=1.2 / dt,
                      sponge_u=(10.0, 0.0, 0.0), sponge_xw=20e3, sponge_yw=10e3),
        num=NumSpec(dt=dt, scheme=scheme),
        steps=int(round(8 * 3600 / dt)), background="stratified", T0=293.15, N=0.01, U=10.0, seed=6)


def hill_large(rotating=True, nx=50, ny=50, nz=50, degree=4, scheme=R2):
    """Larger-scale flow over the bell mountain of Sec. 4.3: a 240 x 240 x 30 km
    Gal-Chen box over h0 / (1 + r^2/a^2) (h0 = 100 m, a = 10 km, centre
    (120, 120) km), periodic in x and y; isothermal hydrostatic background
    T = 250 K (N = g / sqrt(cp T) = 0.0196), uniform wind U = 10 m/s along x;
    Rayleigh damping in the first and last 60 km of x and y and the top 14 km,
    lambda*dt = 1.2; 50^3 elements at r = 4, dt = 4 s, 8 h; f = 1e-4 (rotating
    run) or 0, the geostrophic pressure correction left out as for the
    benchmark hill."""
    dt = 4.0
    return Workload(
        name="hill_large%s_%dx%dx%d_r%d" % ("_rotating" if rotating else "", nx, ny, nz, degree),
        mesh=MeshSpec(240e3, 240e3, 30e3, nx, ny, nz, degree, terrain=BELL, h0=100.0, a=10e3, xc=120e3, yc=120e3),
        phys=PhysSpec(f=1e-4 if rotating else 0.0, sponge_zB=16e3, sponge_zT=30e3, sponge_lam=1.2 / dt,
                      sponge_u=(10.0, 0.0, 0.0), sponge_xw=60e3, sponge_yw=60e3),
        num=NumSpec(dt=dt, scheme=scheme),
        steps=int(round(8 * 3600 / dt)), background="isothermal", T0=250.0, U=10.0, seed=7)


def igw_slice(nx=300, nz=20, degree=4, scheme=R2, planetary=False, dT=0.01):
    """Inertia-gravity waves of Secs. 4.1 and 4.2 in the vertical-slice form (one
    periodic element in y and the slice model, so d/dy = 0 while v stays
    prognostic): isothermal
    T0 = 250 K hydrostatic rest state, Bretherton-transformed perturbation
    T_b = dT exp(-(x - xc)^2 / a^2) sin(pi z / H) with p' = 0, f = 1.03126e-4,
    periodic in x, walls at the bottom and the top, 300 x 20 elements at r = 4.
    Reference channel: 6000 x 10 km, a = 100 km, dt = 0.5 s, 8 h. Planetary
    scale: 60000 x 10 km, a = 1000 km, dt = 10 s, 96 h. The paper does not
    state dT; 0.01 K is used."""
    Lx = 60000e3 if planetary else 6000e3
    a = 1000e3 if planetary else 100e3
    dt = 10.0 if planetary else 0.5
    hours = 96.0 if planetary else 8.0
    return Workload(
        name="igw_slice%s_%dx%d_r%d" % ("_planetary" if planetary else "", nx, nz, degree),
        mesh=MeshSpec(Lx, Lx / nx, 10e3, nx, 1, nz, degree),
        phys=PhysSpec(f=1.03126e-4, slice=1),
        num=NumSpec(dt=dt, scheme=scheme),
        steps=int(round(hours * 3600.0 / dt)), background="isothermal", T0=250.0,
        pert="bretherton", pert_amp=dT, pert_a=a, pert_xc=Lx / 2)


# ------------------------------------------------------------- initial state
def primitive_background(w: Workload, x, y, z):
    """rho, p of the hydrostatic background at points (x, y, z)."""
    if w.background == "isothermal":
        delta = GRAV / (RGAS * w.T0)
        p = P_REF * np.exp(-delta * z)
        rho = p / (RGAS * w.T0)
        return rho, p
    N2 = w.N * w.N
    exner = 1.0 + GRAV * GRAV / (CP * w.T0 * N2) * (np.exp(-N2 * z / GRAV) - 1.0)
    p = P_REF * exner ** (CP / RGAS)
    theta = w.T0 * np.exp(N2 * z / GRAV)
    rho = p / (RGAS * theta * exner)
    return rho, p


def initial_state(w: Workload, coords):
    """Conserved variables [5][E][Np] at node coordinates coords [3][E][Np].

    The potential-temperature perturbations keep the pressure and recompute
    the density; the Bretherton perturbation of Sec. 4.1 adds the linear
    density perturbation rho' = -exp(-delta z / 2) rho_s T_b / T0 at p' = 0. The optional noise multiplies rho and rho*E by (1 + eps xi)
    and adds eps*xi m/s to each velocity component (xi ~ U[-1, 1) drawn per
    field, element and node in that order from numpy default_rng(seed))."""
    x, y, z = coords
    rho, p = primitive_background(w, x, y, z)
    if w.pert == "bretherton":
        delta = GRAV / (RGAS * w.T0)
        rho_s = P_REF / (RGAS * w.T0)
        Tb = w.pert_amp * np.exp(-((x - w.pert_xc) / w.pert_a) ** 2) * np.sin(np.pi * z / w.mesh.Lz)
        rho = rho - np.exp(-0.5 * delta * z) * rho_s * Tb / w.T0
    elif w.pert != "none":
        if w.pert == "gauss":
            r2 = (x - w.pert_xc) ** 2 + (y - w.pert_yc) ** 2 + (z - w.pert_zc) ** 2
            dth = w.pert_amp * np.exp(-r2 / w.pert_a ** 2)
        elif w.pert == "igw":
            dth = w.pert_amp * np.sin(np.pi * z / w.mesh.Lz) / (1.0 + (x - w.pert_xc) ** 2 / w.pert_a ** 2)
        else:
            raise ValueError(w.pert)
        exner = (p / P_REF) ** (RGAS / CP)
        theta = p / (rho * RGAS * exner) + dth
        rho = p / (RGAS * theta * exner)
    u = np.zeros((3,) + x.shape)
    u[0] = w.U
    q = np.empty((5,) + x.shape)
    if w.noise > 0.0:
        xi = np.random.default_rng(w.seed).uniform(-1.0, 1.0, size=(5,) + x.shape)
        u = u + w.noise * xi[1:4]
        rho = rho * (1.0 + w.noise * xi[0])
    q[0] = rho
    q[1:4] = rho * u
    q[4] = p / (GAMMA - 1.0) + 0.5 * rho * (u * u).sum(0)
    if w.noise > 0.0:
        q[4] *= (1.0 + w.noise * xi[4])
    return q


def random_positive_state(shape, seed, rho0=1.0, p0=1e5, urms=10.0, rel=0.05):
    """A generic smooth-free random state with positive density and pressure:
    rho = rho0 (1 + rel xi), u = urms xi, p = p0 (1 + rel xi)."""
    g = np.random.default_rng(seed)
    rho = rho0 * (1.0 + rel * g.uniform(-1, 1, shape))
    u = urms * g.uniform(-1, 1, (3,) + tuple(shape))
    p = p0 * (1.0 + rel * g.uniform(-1, 1, shape))
    q = np.empty((5,) + tuple(shape))
    q[0] = rho
    q[1:4] = rho * u
    q[4] = p / (GAMMA - 1.0) + 0.5 * rho * (u * u).sum(0)
    return q


def conserved_from_primitive(rho, u, p):
    q = np.empty((5,) + np.shape(rho))
    q[0] = rho
    q[1:4] = rho * u
    q[4] = p / (GAMMA - 1.0) + 0.5 * rho * (u * u).sum(0)
    return q


# ------------------------------------------------------------ served ensemble
@dataclass
class Request:
    arrival_s: float
    workload: Workload
    steps: int


def served_trace(n_requests=64, rate_per_s=2.0, elem_min=2000, elem_max=200000, degrees=(2, 3, 4), steps=50,
                 seed=5):
    """Ensemble requests with Poisson arrivals (exponential gaps of mean
    1/rate). Each member is, with probability 1/2, a rotating IGW channel
    (the channel's physics and 25 x 25 x 1 km elements, nz = 10, nx = 3 ny,
    ny = round(sqrt(E / 30))) or an orography member (the orography box's
    physics and 0.9375 x 0.9375 x 0.833 km elements, nz = 24, nx = ny =
    round(sqrt(E / 24)), the hill at the centre), with E uniform in
    [elem_min, elem_max] and the degree drawn from `degrees`: the element sizes,
    and with them the Courant numbers, are those of the two workloads. Each
    member has its own seeded potential-temperature perturbation, amplitude
    0.01 K x (1 + 0.1 xi) with its centre moved by up to 5 % of the domain."""
    g = np.random.default_rng(seed)
    t, out = 0.0, []
    for k in range(n_requests):
        t += g.exponential(1.0 / rate_per_s)
        E = g.uniform(elem_min, elem_max)
        r = int(g.choice(degrees))
        amp = 0.01 * (1.0 + 0.1 * g.uniform(-1.0, 1.0))
        jx, jy = g.uniform(-0.05, 0.05, 2)
        if g.uniform() < 0.5:
            ny = max(2, int(round(np.sqrt(E / 30.0))))
            w = igw_channel(nx=3 * ny, ny=ny, nz=10, degree=r)
            w.mesh.Lx, w.mesh.Ly = 25e3 * 3 * ny, 25e3 * ny
            w.pert_xc = w.mesh.Lx * (0.5 + jx)
            w.pert_a = min(100e3, 0.1 * w.mesh.Lx)
            w.pert_amp = amp
        else:
            n = max(3, int(round(np.sqrt(E / 24.0))))
            w = orography(nx=n, ny=n, nz=24, degree=r)
            L = 0.9375e3 * n
            w.mesh.Lx = w.mesh.Ly = L
            w.mesh.xc = w.mesh.yc = L / 2
            w.pert, w.pert_amp, w.pert_a = "gauss", amp, 2e3
            w.pert_xc, w.pert_yc, w.pert_zc = L * (0.5 + jx), L * (0.5 + jy), 2e3
        w.seed = 1000 + k
        w.name += "_m%d" % k
        out.append(Request(t, w, steps))
    return out

"""Seeded synthetic inputs for the hybrid thermal pseudo-potential LB step.

This module is the one thing the GPU library and the oracle share: it builds
scenario dictionaries (parameters, initial density and temperature fields, and
nucleation-site descriptors) from fixed recipes and numpy PCG64 seeds.  It holds
none of the method's arithmetic: no equation of state, no collision, no stencil.

Parameter values follow Sec. 3.1 and Sec. 4.2 of Hu & Liu (arXiv:1812.10375):
a = 3/49, b = 2/21, R = 1, sigma = 0.107, T_s = 0.86 Tc, c_v = 6, k = 0.1,
nu_l = 0.1 and nu_v = 0.5/3 (tau = 3 nu + 1/2), heater rho_w = 3 rho_l,
lambda_w = 3 lambda_l, c_v,w = c_v,l, wall strength G_w = 0.3.  The acentric factor
omega = 0.344 is not printed in the paper; it is the value that, with the rest of
Sec. 3.1, gives the coexistence densities the paper quotes.

Literal thermodynamic constants below are inputs, not computed here:
  TC      critical temperature fixed by a, b, R (Sec. 3.1)
  RHO_L/V Maxwell coexistence densities at 0.86 Tc
The oracle's test-suite pins all three against the equation of state.
"""
import numpy as np

A = 3.0 / 49.0
B = 2.0 / 21.0
R = 1.0
OMEGA = 0.344
TC = 0.10938300611120136
T_SAT = 0.86 * TC
RHO_L = 6.498945763342
RHO_V = 0.3796789994107
SIGMA = 0.107
CV = 6.0
K_DIFF = 0.1
TAU_L = 0.8   # nu_l = 0.1
TAU_V = 1.0   # nu_v = 0.5/3
GW0 = 0.3

PRECISIONS = ("f32", "f64")


def base_params(**kw):
    """Parameters shared by every scenario; keyword arguments override."""
    p = dict(
        nx=64, ny=64, heater_rows=0, n_sub=1,
        top_bc="wall", bottom_tbc="dirichlet", top_tbc="dirichlet", flags=(),
        a=A, b=B, R=R, omega=OMEGA, T_sat=T_SAT, G=-1.0, sigma=SIGMA,
        tau_l=TAU_L, tau_v=TAU_V, s_e=0.8, s_zeta=0.8, s_q=1.1,
        rho_l=RHO_L, rho_v=RHO_V,
        cv=CV, k=K_DIFF, rho_w=3.0 * RHO_L, cv_w=CV, lambda_w=3.0 * RHO_L * CV * K_DIFF,
        g=0.0, T_bottom=T_SAT, T_top=T_SAT, q_bottom=0.0, Gw0=0.0, Gw_top=0.0,
        sites=np.zeros((0, 3)), precision="f64", steps=100,
    )
    p.update(kw)
    return p


def layered_density(nx, ny, n_liquid, rng=None, perturb=0.0):
    """Liquid rows 0..n_liquid-1 at RHO_L, vapour above at RHO_V (sharp step),
    plus an optional uniform perturbation U(-perturb, perturb) from ``rng``."""
    rho = np.full((ny, nx), RHO_V)
    rho[:n_liquid, :] = RHO_L
    if perturb:
        rho = rho + rng.uniform(-perturb, perturb, size=rho.shape)
    return rho


def sample_sites(rng, nx, n_sites, min_spacing, width, gmins=(0.0, -0.3, -0.6)):
    """Site centres by rejection sampling of U{0..nx-1} with a periodic minimum
    spacing; minima cycle through ``gmins`` from left to right (Sec. 4.2)."""
    centres = []
    tries = 0
    while len(centres) < n_sites:
        tries += 1
        if tries > 100000:
            raise ValueError("cannot place %d sites with spacing %d on %d columns"
                             % (n_sites, min_spacing, nx))
        c = int(rng.integers(0, nx))
        if all(min(abs(c - o), nx - abs(c - o)) >= min_spacing for o in centres):
            centres.append(c)
    centres.sort()
    return np.array([[c, width, gmins[k % len(gmins)]] for k, c in enumerate(centres)],
                    dtype=np.float64)


def regular_sites(nx, spacing, width, gmins=(0.0, -0.3, -0.6)):
    """Evenly spaced sites: centres at spacing/2 + k*spacing, k < nx // spacing."""
    n = max(1, nx // spacing)
    return np.array([[spacing / 2.0 + k * spacing, width, gmins[k % len(gmins)]] for k in range(n)],
                    dtype=np.float64)


def interface_conduction(nx=8, ny=256, exact_energy=True, steps=5000, precision="f64"):
    """1-D heat conduction across a flat liquid-vapour interface (Sec. 3.2 analogue,
    y-oriented): walls at both ends held at 0.87 Tc and 0.85 Tc, liquid lower half,
    vapour upper half, EOS temperature frozen at T_s, no gravity, neutral walls."""
    flags = ("freeze_eos_T", "no_advection", "no_latent") if exact_energy else ("freeze_eos_T",)
    return base_params(
        name="interface_conduction_%dx%d" % (nx, ny), nx=nx, ny=ny, heater_rows=0,
        top_bc="wall", bottom_tbc="dirichlet", top_tbc="dirichlet", flags=flags,
        T_bottom=0.87 * TC, T_top=0.85 * TC, Gw0=0.0, Gw_top=0.0, g=0.0,
        rho0=layered_density(nx, ny, ny // 2), T0=np.full((ny, nx), T_SAT),
        precision=precision, steps=steps)


def film_evaporation(nx=256, ny=256, film=40, superheat=0.05, seed=2, steps=20000,
                     precision="f32"):
    """Liquid film on a heated wall (Sec. 3.3 family): Dirichlet wall at
    T_s + superheat*Tc below row 0, film of ``film`` rows, vapour above, constant
    pressure top at rho_v, seeded +-1e-4 density perturbation."""
    rng = np.random.default_rng(seed)
    return base_params(
        name="film_evaporation_%dx%d" % (nx, ny), nx=nx, ny=ny, heater_rows=0,
        top_bc="const_pressure", bottom_tbc="dirichlet", top_tbc="zero_grad",
        T_bottom=T_SAT + superheat * TC, Gw0=GW0, g=0.0,
        rho0=layered_density(nx, ny, film, rng, 1e-4), T0=np.full((ny, nx), T_SAT),
        precision=precision, steps=steps, seed=seed)


def film_evaporation_flux(ratio=1.0, q=2e-4, nx=20, ny=100, film=50, wall=20, n_sub=5, precision="f64",
                          isotropic=False):
    """Film evaporation driven by a heat flux through a wall (Sec. 3.3): a wall of
    ``wall`` rows with rho_w = 3 rho_l, c_v,w = c_v and lambda_w = ratio * lambda_l
    receives q through its bottom; a liquid film of ``film`` rows lies on it, vapour
    above, with a constant-pressure top at rho_v; neutral wall, no gravity, everything
    starts at T_s.  ``n_sub`` energy sub-steps per LB step (Eq. 27) keep the RK4 update
    stable in the more conductive walls.  The default sizes are the paper's (20 x 120
    with the wall)."""
    sc = base_params(
        name="film_flux_r%g_%dx%d+%d" % (ratio, nx, ny, wall), nx=nx, ny=ny, heater_rows=wall, n_sub=n_sub,
        top_bc="const_pressure", bottom_tbc="flux", top_tbc="zero_grad", q_bottom=q,
        rho_w=3.0 * RHO_L, cv_w=CV, lambda_w=ratio * RHO_L * CV * K_DIFF, Gw0=0.0,
        flags=("diff_isotropic",) if isotropic else (),
        rho0=layered_density(nx, ny, film), T0=np.full((wall + ny, nx), T_SAT), precision=precision)
    return sc


def pool_boiling(nx=1024, ny=1024, heater_rows=25, superheat=0.10, g=3e-5, n_sites=8,
                 min_spacing=64, site_width=4.0, liquid_fraction=0.7, seed=3, steps=100000,
                 precision="f32", site_spacing=None, Gw0=GW0):
    """Pool boiling on a conjugate heater with nucleation sites (Sec. 4.2 family):
    heater rows below the fluid, its bottom held at T_s + superheat*Tc, convective
    outlet at the top, gravity along -y, liquid filling the lower fraction.  Sites are
    sampled with a minimum spacing, or evenly spaced when ``site_spacing`` is given."""
    rng = np.random.default_rng(seed)
    if site_spacing:
        sites = regular_sites(nx, int(site_spacing), site_width)
    elif n_sites:
        sites = sample_sites(rng, nx, n_sites, min_spacing, site_width)
    else:
        sites = np.zeros((0, 3))
    n_liq = int(round(liquid_fraction * ny))
    return base_params(
        name="pool_boiling_%dx%d" % (nx, ny), nx=nx, ny=ny, heater_rows=heater_rows,
        top_bc="convective", bottom_tbc="dirichlet", top_tbc="zero_grad",
        T_bottom=T_SAT + superheat * TC, Gw0=Gw0, g=g, sites=sites,
        rho0=layered_density(nx, ny, n_liq), T0=np.full((heater_rows + ny, nx), T_SAT),
        precision=precision, steps=steps, seed=seed)


BATCH_SIZES = ((256, 256), (512, 256), (512, 512), (1024, 512))  # (nx, ny)


def batched_pool_boiling(n=48, seed=7, heater_rows=25, precision="f32", steps=50000, liquid_fraction=1.0):
    """Independent pool-boiling domains of uneven sizes for the batched step: sizes drawn
    from BATCH_SIZES, superheats from U(0.02, 0.30) Tc, 2-12 nucleation sites per domain
    (periodic minimum spacing nx / (2 n_sites), at least 8 columns), every domain seeded
    from one generator.  The pools start filled with liquid, as the paper's boiling runs
    do (Sec. 4.2)."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        nx, ny = BATCH_SIZES[int(rng.integers(0, len(BATCH_SIZES)))]
        superheat = float(rng.uniform(0.02, 0.30))
        n_sites = int(rng.integers(2, 13))
        sc = pool_boiling(nx=nx, ny=ny, heater_rows=heater_rows, superheat=superheat,
                          n_sites=n_sites, min_spacing=max(8, nx // (2 * n_sites)),
                          seed=int(rng.integers(0, 2**31)), precision=precision, steps=steps,
                          liquid_fraction=liquid_fraction)
        sc["name"] = "batch%02d_%s" % (i, sc["name"])
        out.append(sc)
    return out


# Surrogate network parameter vector of one member (row-major; a layer computes
# z = h W + b for a row vector h): W1[4][128], b1[128], W2[128][128], b2[128],
# W3[128][2], b3[2].
MLP_SHAPES = ((4, 128), (128,), (128, 128), (128,), (128, 2), (2,))


def mlp_init_params(seed, members):
    """Seeded initial weights of an ensemble: weights uniform within the Glorot bounds
    +-sqrt(6 / (fan_in + fan_out)), biases zero; returns members x 17410 float64."""
    rng = np.random.default_rng(seed)
    rows = []
    for _ in range(members):
        parts = []
        for shape in MLP_SHAPES:
            if len(shape) == 2:
                lim = np.sqrt(6.0 / (shape[0] + shape[1]))
                parts.append(rng.uniform(-lim, lim, size=shape).ravel())
            else:
                parts.append(np.zeros(shape))
        rows.append(np.concatenate(parts))
    return np.array(rows)


def static_droplet(nx, ny, radius, seed=None, precision="f64", bubble=False):
    """Fully periodic-in-x box with walls, a circular drop (or bubble) in the middle."""
    yy, xx = np.mgrid[0:ny, 0:nx]
    d = np.sqrt((xx + 0.5 - nx / 2) ** 2 + (yy + 0.5 - ny / 2) ** 2)
    inside = d < radius
    rho = np.where(inside, RHO_V if bubble else RHO_L, RHO_L if bubble else RHO_V)
    return base_params(
        name="static_%s_r%g" % ("bubble" if bubble else "drop", radius), nx=nx, ny=ny,
        flags=("freeze_eos_T", "no_advection", "no_latent"), rho0=rho.astype(np.float64),
        T0=np.full((ny, nx), T_SAT), precision=precision)


def sessile_drop(nx, ny, radius, Gw, precision="f64"):
    """Half-disc of liquid resting on the bottom wall (wall strength Gw), vapour around,
    isothermal, for the contact-angle check of Sec. 4.2."""
    yy, xx = np.mgrid[0:ny, 0:nx]
    d = np.sqrt((xx + 0.5 - nx / 2) ** 2 + (yy + 0.5) ** 2)
    rho = np.where(d < radius, RHO_L, RHO_V)
    return base_params(
        name="sessile_Gw%g" % Gw, nx=nx, ny=ny, top_bc="wall",
        flags=("freeze_eos_T", "no_advection", "no_latent"), Gw0=Gw, Gw_top=0.0,
        rho0=rho.astype(np.float64), T0=np.full((ny, nx), T_SAT), precision=precision)


def workloads():
    """The named full-size workloads."""
    return {
        "interface_conduction_8x256": interface_conduction(),
        "film_evaporation_256x256": film_evaporation(),
        "pool_boiling_1024x1024": pool_boiling(),
    }

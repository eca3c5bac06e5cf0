"""Closed forms of the discrete model's large-scale behaviour, used to pin the
step loop to physics it must reproduce (the diffusion regime the paper's
introduction contrasts with transport, Sec. 1, and the random walk of
multiple scattering, Sec. 3.1).

Test infrastructure only (see the package docstring)."""
import math


def persistent_walk_msd(m, ell, lam, omega_sq):
    """Mean squared displacement along one axis after m steps of a random walk
    with step length ell, direction kept from step to step with correlation
    lam = <cos> between successive directions, and <Omega_i^2> = omega_sq:
        <X^2> = ell^2 omega_sq [m (1 + lam)/(1 - lam) - 2 lam (1 - lam^m)/(1 - lam)^2].
    (Sum of m unit steps with exponentially decaying correlation lam^|i-j|.)"""
    return ell * ell * omega_sq * (m * (1.0 + lam) / (1.0 - lam)
                                   - 2.0 * lam * (1.0 - lam ** m) / (1.0 - lam) ** 2)


def step_correlation(a, b, g_p):
    """Correlation of successive directions of a surviving photon in the
    collision update: unscattered with probability a/(a+b), otherwise redrawn
    from the discrete phase matrix whose mean cosine is g_p."""
    return (a + b * g_p) / (a + b)


def walk_diffusion_coefficient(ell, dt, lam):
    """Diffusion coefficient of the persistent walk in 3-D:
    D = ell^2 (1 + lam) / (6 dt (1 - lam))."""
    return ell * ell * (1.0 + lam) / (6.0 * dt * (1.0 - lam))


def cube_decay_rate(D, L_side, v, survival_per_step, dt, extrapolation=True):
    """Late-time decay rate of the total photon number in a cube of side L with
    absorbing walls in the diffusion approximation: the fundamental mode
    sin(pi x/L_e) sin(pi y/L_e) sin(pi z/L_e) decays at 3 D (pi/L_e)^2, plus the
    absorption rate -ln(survival)/dt.  L_e = L + 4 D/v adds the extrapolation
    length 2D/v at each wall."""
    L_e = L_side + (4.0 * D / v if extrapolation else 0.0)
    return 3.0 * D * (math.pi / L_e) ** 2 - math.log(survival_per_step) / dt

"""Threshold speed c* of travelling fronts by shooting (TEST INFRASTRUCTURE ONLY).

The appendix (after Malaguti and Marcelli) ties travelling fronts of
u_t = (D(u) u_x)_x + g(u) on [0, umax] (D, g vanishing at 0 and umax, positive
in between) to solutions z(u) < 0 of

    dz/du = -c - D(u) g(u) / z,   z(0+) = z(umax-) = 0,

and the threshold c* is the infimum of the c that admit one (sets
defAchi0 / defA0; the paper bounds it by c-bar, Sec. 4.1).  At c = c* the
front is sharp: its z leaves u = 0 along z = -c u + h2 u^2 / (2 c) + ...
(h2 = lim D g / u^2).  Followed upwards from there, the trajectory of a
c < c* returns to z = 0 before u reaches umax, and that of a c > c* arrives at
u = umax with z < 0; c* separates the two and follows by bisection.  The
integration is scipy's adaptive DOP853 with a terminal event at z = 0.
"""
from scipy.integrate import solve_ivp


def _below_threshold(c, h, h2, umax, eps):
    """True when the sharp-start trajectory of speed c returns to z = 0 before
    u = umax (1 - eps), i.e. c < c*."""
    u0 = eps * umax
    z0 = -c * u0 + h2 * u0 * u0 / (2.0 * c)

    def rhs(u, z):
        return [-c - h(u) / z[0]]

    def hit_zero(u, z):
        return z[0]
    hit_zero.terminal = True
    hit_zero.direction = 1
    u1 = umax * (1.0 - eps)
    sol = solve_ivp(rhs, (u0, u1), [z0], method="DOP853", rtol=1e-10,
                    atol=1e-14 * umax * c, events=hit_zero)
    # below the threshold the trajectory meets z = 0 early (the event fires, or
    # the step size collapses as z -> 0 with D g > 0 and the solver stops)
    return sol.status != 0 or sol.t[-1] < u1 or sol.y[0, -1] >= 0.0


def threshold_speed(D, g, umax, h2, c_hi, eps=1e-6, iters=50):
    """c* of u_t = (D u_x)_x + g on [0, umax]; h2 = lim D g / u^2 at u = 0,
    and c_hi must exceed c*."""
    h = lambda u: D(u) * g(u)
    lo, hi = 0.0, float(c_hi)
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        if _below_threshold(mid, h, h2, umax, eps):
            lo = mid
        else:
            hi = mid
        if hi - lo <= 1e-10 * hi:
            break
    return 0.5 * (lo + hi)


def cstar(n0, chi, sigma0=1.0):
    """c*(n0, chi0) for the scalar equation eq. scalar-eq-b-re of Sec. 4.1:
    D = sigma0 D-tilde(b, chi0) (eq. D-tilde), g = n0 b (1 - b / n0)
    (eq. reac-term), on [0, n0]; near b = 0, D g = sigma0 n0^2 b^2 + ..."""
    from .cbar import cbar
    Dt = lambda b: sigma0 * n0 * b * (1.0 - b / n0) * (1.0 + chi * b)
    g = lambda b: n0 * b * (1.0 - b / n0)
    return threshold_speed(Dt, g, n0, sigma0 * n0 * n0, 1.05 * cbar(n0, chi, sigma0))

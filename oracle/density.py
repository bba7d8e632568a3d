"""Choice of the density operator A(rho, v) of Sec. 3.1 eq:Conv: the
semi-Lagrangian one ("sl") or the paper's upwind Taylor exponential
("upwind", eq:Adv).  Sec. 4.1 allows any operator whose partials in rho and
v are available; these three calls are all the density subproblem, the
re-simulation and the adjoints use.

Test infrastructure: only the tests, the smoke check and the benchmark's CPU
baseline use this package."""
from . import advect, upwind

KINDS = ("sl", "upwind")


def fwd(g, rho, v, dt, kind="sl"):
    """A(rho, v)."""
    if kind == "sl":
        return advect.advect_scalar(g, rho, v, dt)
    assert kind == "upwind", kind
    return upwind.advect_up(g, rho, v, dt)


def adj_rho(g, mu, rho, v, dt, kind="sl"):
    """(dA(rho, v)/drho)^T mu."""
    if kind == "sl":
        return advect.advect_scalar_T(g, mu, v, dt)
    assert kind == "upwind", kind
    return upwind.advect_up_T(g, mu, rho, v, dt)


def adj_v(g, mu, rho, v, dt, kind="sl"):
    """(dA(rho, v)/dv)^T mu."""
    if kind == "sl":
        return advect.advect_scalar_dv_T(g, mu, rho, v, dt)
    assert kind == "upwind", kind
    return upwind.advect_up_dv_T(g, mu, rho, v, dt)

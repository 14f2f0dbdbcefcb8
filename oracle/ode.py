"""Integrators of the flow ODE dx/dt = v(x, t) — oracle side.

The paper samples the learned vector field with Euler integration and lets the user set
the number of steps (Sec. 2.2; default 50 in App. C). Readings used here: noise sits at
t0 = 0 and data at t1 = 1 (the rectified-flow / flow-matching convention of the
references the paper cites for the method); the grid is uniform, t_k = t0 + k h with
h = (t1 - t0)/K; Euler evaluates v at the left end of each step. The workloads also ask
for classic fourth-order Runge-Kutta, which the paper does not use; its stages sit at
t_k, t_k + h/2, t_k + h/2 and t_k + h with weights 1/6, 2/6, 2/6, 1/6. For comparisons of
integrators at an equal evaluation budget (the paper: the step count trades generation
speed for quality), the explicit midpoint rule is offered as well: k1 = v(x, t_k),
x <- x + h v(x + (h/2) k1, t_k + h/2), two evaluations per step.
"""

import numpy as np

EULER, RK4, MIDPOINT = 0, 1, 2


def stage_times(scheme, n_steps, t0=0.0, t1=1.0):
    """List of (t, step) for every velocity evaluation, in evaluation order."""
    h = (t1 - t0) / n_steps
    out = []
    for k in range(n_steps):
        tk = t0 + k * h
        if scheme == EULER:
            out.append(tk)
        elif scheme == MIDPOINT:
            out += [tk, tk + 0.5 * h]
        else:
            out += [tk, tk + 0.5 * h, tk + 0.5 * h, tk + h]
    return out


def integrate(v, x0, scheme, n_steps, t0=0.0, t1=1.0):
    """Integrate dx/dt = v(x, t) from x0 at t0 to t1 in n_steps uniform steps."""
    if n_steps < 1:
        raise ValueError("n_steps must be >= 1")
    h = (t1 - t0) / n_steps
    x = np.array(x0, copy=True)
    for k in range(n_steps):
        tk = t0 + k * h
        if scheme == EULER:
            x = x + h * v(x, tk)
        elif scheme == MIDPOINT:
            k1 = v(x, tk)
            x = x + h * v(x + 0.5 * h * k1, tk + 0.5 * h)
        elif scheme == RK4:
            k1 = v(x, tk)
            k2 = v(x + 0.5 * h * k1, tk + 0.5 * h)
            k3 = v(x + 0.5 * h * k2, tk + 0.5 * h)
            k4 = v(x + h * k3, tk + h)
            x = x + (h / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4)
        else:
            raise ValueError(f"unknown scheme {scheme}")
    return x

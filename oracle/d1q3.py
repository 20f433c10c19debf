"""TEST INFRASTRUCTURE ONLY -- the one-dimensional toy of the paper's introduction.

Kaushal, Succi & Ansumali (arXiv:2210.10377), Sec. I, Eq. lbb1-lbb4 and Fig. 4 (the
D1Q3 lattice with boundary node X_1): a three-velocity lattice (c = 0, +1, -1) on nodes
X_1 ... X_n, a bounce-back wall half-way to the left of X_1, and the momentum balance of
the control volume {X_1, X_2, ...} over one collide-stream step.  The paper does not
print the D1Q3 weights; the standard ones (2/3, 1/6, 1/6, theta0 = 1/3) are used.

Pure Python on a handful of nodes; the right end is far enough away that nothing from
it reaches the control volume within the steps taken (the semi-infinite control volume
of the toy).
"""
from __future__ import annotations

C = (0, 1, -1)
W = (2.0 / 3.0, 1.0 / 6.0, 1.0 / 6.0)
THETA0 = 1.0 / 3.0


def equilibrium(rho, u):
    """Second-order equilibrium (Sec. II) on the D1Q3 lattice."""
    return [W[i] * rho * (1.0 + C[i] * u / THETA0 + ((C[i] * u) ** 2 - THETA0 * u * u)
                          / (2.0 * THETA0 * THETA0)) for i in range(3)]


def collide(f, beta):
    """Eq. lbb1, first line: f~ = f + 2 beta (f^eq - f)."""
    rho = sum(f)
    u = sum(C[i] * f[i] for i in range(3)) / rho
    feq = equilibrium(rho, u)
    return [f[i] + 2.0 * beta * (feq[i] - f[i]) for i in range(3)]


def momentum(nodes, upto):
    """J_X = sum over the first ``upto`` nodes of sum_i c_i f_i (the global momentum of
    the toy's control volume)."""
    return sum(C[i] * nodes[q][i] for q in range(upto) for i in range(3))


def step(nodes, beta, collided_return: bool):
    """One collide-then-stream step (Eq. lbb1).  The wall left of X_1 returns either the
    post-collision population f~_{-1}(X_1, t) (collided_return=True, the choice of
    algorithm B) or the un-collided f_{-1}(X_1, t) (the naive choice of algorithm A).
    Returns (new_nodes, post_collision_nodes)."""
    n = len(nodes)
    post = [collide(f, beta) for f in nodes]
    new = [[0.0, 0.0, 0.0] for _ in range(n)]
    for q in range(n):
        new[q][0] = post[q][0]
        if q + 1 < n:
            new[q + 1][1] = post[q][1]
        if q - 1 >= 0:
            new[q - 1][2] = post[q][2]
    new[0][1] = post[0][2] if collided_return else nodes[0][2]
    new[n - 1][2] = post[n - 1][2]  # far right end: reflect in place (never reached)
    return new, post

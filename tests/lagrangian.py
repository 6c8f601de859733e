"""Equations of motion from energies alone, for pinning the oracle's dynamics.

Given the positions of point masses and the angles of rigid bodies as
functions of the generalised coordinates q, the kinetic energy is
T = sum m |dp/dt|^2 / 2 + sum I (dphi/dt)^2 / 2 and the Euler-Lagrange
equations read M(q) qdd + (dM/dt) qd - dT/dq + dV/dq = Q. Here the velocity
Jacobians come from complex-step differentiation (exact to rounding) and the
remaining derivatives from central differences, so nothing of the oracle's
closed-form equations is reused.
"""
import numpy as np


def _jac(fun, q, k, h=1e-30):
    qc = np.array(q, dtype=complex)
    qc[k] += 1j * h
    return np.imag(np.asarray(fun(qc))) / h


class Body:
    """Point masses (mass, position fn) and rotating bodies (inertia, angle fn)."""

    def __init__(self, masses, inertias, g_vec):
        self.masses = masses      # list of (m, p(q) -> 2-vector)
        self.inertias = inertias  # list of (I, phi(q) -> angle)
        self.g_vec = np.asarray(g_vec, dtype=float)

    def mass_matrix(self, q):
        n = len(q)
        M = np.zeros((n, n))
        for m, p in self.masses:
            J = np.stack([_jac(p, q, k) for k in range(n)], axis=1)  # 2 x n
            M += m * J.T @ J
        for inertia, phi in self.inertias:
            j = np.array([_jac(phi, q, k) for k in range(n)])
            M += inertia * np.outer(j, j)
        return M

    def kinetic(self, q, qd):
        return 0.5 * qd @ self.mass_matrix(q) @ qd

    def potential(self, q):
        return sum(-m * self.g_vec @ np.real(np.asarray(p(np.asarray(q, dtype=complex))))
                   for m, p in self.masses)

    def accel(self, q, qd, Q, h=1e-5):
        q = np.asarray(q, float)
        qd = np.asarray(qd, float)
        n = len(q)
        M = self.mass_matrix(q)
        mdot_qd = np.zeros(n)
        dTdq = np.zeros(n)
        dVdq = np.zeros(n)
        for k in range(n):
            e = np.zeros(n)
            e[k] = h
            dM = (self.mass_matrix(q + e) - self.mass_matrix(q - e)) / (2 * h)
            mdot_qd += (dM @ qd) * qd[k]
            dTdq[k] = 0.5 * qd @ dM @ qd
            dVdq[k] = (self.potential(q + e) - self.potential(q - e)) / (2 * h)
        rhs = np.asarray(Q, float) + dTdq - dVdq - mdot_qd
        return np.linalg.solve(M, rhs)

    def energy(self, q, qd):
        return self.kinetic(np.asarray(q, float), np.asarray(qd, float)) + self.potential(q)

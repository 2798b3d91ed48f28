"""Error bounds for the complex64 path (FP32 state, matrices composed in FP64
and rounded once, FP64 readouts).

Rigorous bound (standard floating-point model, unit roundoff u = 2^-24,
gamma_m = m u / (1 - m u), Higham, Accuracy and Stability of Numerical
Algorithms, inner-product bound): a dense op of k qubits computes each output
as a real inner product of 2^(k+1) terms, so its error is at most
    eps_k = (sqrt(2) gamma_(2^(k+1)) + u) * 2^(k/2)
times the 2-norm of its input (the u term covers the single rounding of the
matrix to FP32, the 2^(k/2) bounds the 2-norm of |U| for unitary U); a
diagonal op costs eps_diag = sqrt(2) gamma_2 + u; a +-1 diagonal costs 0.
A single-qubit gate split into phase * rotation * phase has two diagonal ops
and one rotation run as two shears after a scaling diag(c, 1/c) that joins the
diagonal before it (c = cos theta >= 1/sqrt 2, shear coefficients |beta| <=
1/2, |alpha| <= 1).  The shears undo the scaling exactly (S_alpha S_beta =
Rot Lambda^-1), and every rounding error made while a component carries its
scale factor is proportional to that component, so after the shears it
counts at the unscaled size: the diagonal keeps its eps_diag.  For a pair
(x0, x1) of norm rho: z0 = y0 + beta y1 has |z0| <= rho, its FMA rounding
<= u rho and the rounding of beta <= |beta| u |y1| <= u rho / sqrt 2; z1 = y1 +
alpha z0 takes z0's error times |alpha| <= 1, its own FMA rounding and the
rounding of alpha, each <= u rho.  The pair's error is at most
sqrt(1.71^2 + 3.71^2) u rho = 4.08 u rho, so
    eps_rot = 4.08 u (1 + 1e-4) + 2e-14
per rotated qubit (the last term covers the FP64 factorisation).  Errors of
successive ops add to first order:
    ||psi_c64 - psi_exact||_2 <= sum over ops of eps_op,
and max|delta amp| <= ||delta||_2, 1 - fidelity <= ||delta||_2^2.

Typical estimate (probabilistic rounding-error model: every rounding error is
an independent, mean-zero relative perturbation, uniform on [-u, u], so of
variance u^2 / 3 -- the model behind the square-root growth of Higham and
Mary, "A new approach to probabilistic rounding error analysis", SIAM J. Sci.
Comput. 41 (2019)).  An output component that passes through rho roundings of
values of about its own size gets an error of standard deviation
u sqrt(rho / 3) relative to it; summed over the components of a unitary op
the error's 2-norm is about u sqrt(rho / 3) ||x||.  rho per op kind:
  dense k:   the inner product of m = 2^(k+1) real terms accumulates m
             roundings of partial sums that grow like a random walk
             (mean square (j / m) of the final value at step j: m / 2 in
             total), plus one rounding of each coefficient (1 in total):
             rho = 2^k + 1;
  diagonal:  one product and one FMA per component plus the coefficient: 3;
  rotation:  two shears: z1 passes through its own FMA, alpha's rounding
             and z0's two (FMA, beta) carried by |alpha| <= 1, z0 through
             two: at most 4 per component;
  +-1 diagonal: exact, 0.
Independent ops add in quadrature: typical = u sqrt(sum_ops rho_op / 3).  The
tests assert measured <= TYPICAL_MULTIPLE * typical (and <= the rigorous
bound): an error ten times the size the model expects fails, while the
rigorous bound alone would let errors thousands of times too large pass.
"""
from __future__ import annotations

import math

U32 = 2.0 ** -24
TYPICAL_MULTIPLE = 10.0


def gamma(m):
    return m * U32 / (1 - m * U32)


def eps_dense(k):
    return (math.sqrt(2) * gamma(2 ** (k + 1)) + U32) * 2 ** (k / 2)


EPS_DIAG = math.sqrt(2) * gamma(2) + U32
EPS_ROT = math.sqrt((1 + 1 / math.sqrt(2)) ** 2 + (3 + 1 / math.sqrt(2)) ** 2) * U32 * (1 + 1e-4) + 2e-14

RHO_DIAG = 3.0
RHO_ROT = 4.0


def rho_dense(k):
    return 2.0 ** k + 1


def bounds_from_counts(ops_dense, ops_diag, ops_rot):
    """(rigorous, typical) for op counts: ops_dense[k] dense ops of k qubits
    (k = 1..5), ops_diag diagonal ops with non-trivial entries, ops_rot
    rotated qubits."""
    rig = sum(ops_dense[k] * eps_dense(k) for k in range(1, 6)) + ops_diag * EPS_DIAG + ops_rot * EPS_ROT
    rho = sum(ops_dense[k] * rho_dense(k) for k in range(1, 6)) + ops_diag * RHO_DIAG + ops_rot * RHO_ROT
    return rig, U32 * math.sqrt(rho / 3.0)


def bound_for(plan):
    """(rigorous, typical) for a complex64 plan, from its op counts."""
    s = plan.stats()
    return bounds_from_counts(s["ops_dense"], s["ops_diag"], s["ops_rot"])


def bound_gbg(circuit):
    """(rigorous, typical) for the gate-by-gate path: one dense op per gate."""
    dense = [0] * 6
    for g in circuit.gates:
        dense[g.k] += 1
    return bounds_from_counts(dense, 0, 0)


def check(measured_l2, rig, typ):
    """Assert measured <= rigorous bound and <= TYPICAL_MULTIPLE x typical."""
    assert measured_l2 <= rig, ("above the rigorous bound", measured_l2, rig)
    assert measured_l2 <= TYPICAL_MULTIPLE * typ, ("above %g x the typical estimate" % TYPICAL_MULTIPLE,
                                                   measured_l2, typ)

"""Seeded synthetic inputs shared by the oracle and the GPU path.

This module only *describes* circuits and observables: gate names, qubit
indices, angles and parameter slots, all drawn from numpy's PCG64 generator.
It builds no gate matrices and applies nothing; each side turns a gate
description into a matrix with its own code.

Gate conventions (qubit k is bit k of the amplitude index, the pairing rule of
Sec. III.A Eq. 5):

* ``op`` is one of ``h x y z s sdg t tdg rx ry rz p u3 cx cz cp swap mat1 mat2``;
* ``qubits`` is a tuple. For ``cx``/``cz``/``cp`` it is ``(control, target)``;
  for ``swap`` and ``mat2`` it is ``(t0, t1)`` where the 4x4 matrix index is
  ``bit(t0) + 2*bit(t1)``;
* ``params`` holds the angles (``rx ry rz p cp``: one, ``u3``: three) or, for
  ``mat1``/``mat2``, the row-major complex matrix flattened to (re, im) pairs;
* ``param_index`` is the slot of a trainable angle (``-1`` when fixed). Only
  ``rx``/``ry``/``rz`` may carry a slot; ``params[0]`` is then the angle used.

Observables are lists of ``(coeff, x_mask, z_mask)`` Pauli strings: bit k of
``x_mask``/``z_mask`` puts X/Z on qubit k, both bits set puts Y there.
"""
from __future__ import annotations

from collections import namedtuple
from typing import List, Sequence, Tuple

import numpy as np

Gate = namedtuple("Gate", "op qubits params param_index")

ONE_QUBIT = ("h", "x", "y", "z", "s", "sdg", "t", "tdg", "rx", "ry", "rz", "p", "u3", "mat1")
TWO_QUBIT = ("cx", "cz", "cp", "swap", "mat2")
PARAMETRIC = ("rx", "ry", "rz")
N_ANGLES = {"rx": 1, "ry": 1, "rz": 1, "p": 1, "cp": 1, "u3": 3}


def gate(op: str, *qubits: int, params: Sequence[float] = (), param_index: int = -1) -> Gate:
    return Gate(op, tuple(int(q) for q in qubits), tuple(float(p) for p in params), int(param_index))


def rng_for(seed: int) -> np.random.Generator:
    """The one generator every input recipe draws from (numpy PCG64)."""
    return np.random.Generator(np.random.PCG64(seed))


# ---------------------------------------------------------------- circuits ---

def random_u3_layers(n: int, depth: int, seed: int, entangler: str = "cx") -> List[Gate]:
    """Layered random circuit: per layer, U3 with three angles ~ U[0, 2pi) on
    every qubit (qubit 0 first), then ``entangler`` on a random perfect matching.

    The matching shuffles the qubits with the seeded generator and pairs
    consecutive entries; for odd ``n`` the last qubit idles that layer. For
    ``cx`` the first entry of each pair is the control.
    """
    if entangler not in ("cx", "cz"):
        raise ValueError("entangler must be 'cx' or 'cz'")
    rng = rng_for(seed)
    out: List[Gate] = []
    for _ in range(depth):
        angles = rng.uniform(0.0, 2.0 * np.pi, size=(n, 3))
        for q in range(n):
            out.append(gate("u3", q, params=angles[q]))
        perm = rng.permutation(n)
        for j in range(n // 2):
            out.append(gate(entangler, int(perm[2 * j]), int(perm[2 * j + 1])))
    return out


def qft(n: int) -> List[Gate]:
    """Textbook quantum Fourier transform on n qubits, qubit n-1 most significant:
    for j = n-1 .. 0: H(j), then CP(2pi / 2^(j-m+1)) on (m, j) for m = j-1 .. 0;
    finally SWAP(q, n-1-q) for q < n // 2."""
    out: List[Gate] = []
    for j in range(n - 1, -1, -1):
        out.append(gate("h", j))
        for m in range(j - 1, -1, -1):
            out.append(gate("cp", m, j, params=(2.0 * np.pi / float(2 ** (j - m + 1)),)))
    for q in range(n // 2):
        out.append(gate("swap", q, n - 1 - q))
    return out


def random_basis_index(n: int, seed: int) -> int:
    """x ~ U{0 .. 2^n - 1}."""
    return int(rng_for(seed).integers(0, 1 << n, dtype=np.uint64))


def hea(n: int, layers: int, thetas: Sequence[float]) -> List[Gate]:
    """Hardware-efficient ansatz: per layer l and qubit q, RY(theta[2(l n + q)])
    then RZ(theta[2(l n + q) + 1]); then CZ(q, q+1) for q = 0 .. n-2."""
    thetas = np.asarray(thetas, dtype=np.float64)
    if thetas.shape != (2 * n * layers,):
        raise ValueError("need 2*n*layers angles")
    out: List[Gate] = []
    for l in range(layers):
        for q in range(n):
            p = 2 * (l * n + q)
            out.append(gate("ry", q, params=(thetas[p],), param_index=p))
            out.append(gate("rz", q, params=(thetas[p + 1],), param_index=p + 1))
        for q in range(n - 1):
            out.append(gate("cz", q, q + 1))
    return out


def hea_params(n: int, layers: int, seed: int) -> np.ndarray:
    """theta ~ U[-pi, pi], 2 n layers of them."""
    return rng_for(seed).uniform(-np.pi, np.pi, size=2 * n * layers)


def with_params(circuit: Sequence[Gate], thetas: Sequence[float]) -> List[Gate]:
    """Copy of ``circuit`` whose trainable gates take their angle from ``thetas``."""
    out = []
    for g in circuit:
        if g.param_index >= 0:
            out.append(Gate(g.op, g.qubits, (float(thetas[g.param_index]),), g.param_index))
        else:
            out.append(g)
    return out


def n_params(circuit: Sequence[Gate]) -> int:
    return 1 + max((g.param_index for g in circuit), default=-1)


# ------------------------------------------------------------- observables ---

def zz_x_chain(n: int, x_coeff: float = 0.5) -> List[Tuple[float, int, int]]:
    """Open chain sum_{i<n-1} Z_i Z_{i+1} + x_coeff * sum_i X_i."""
    terms = [(1.0, 0, (1 << i) | (1 << (i + 1))) for i in range(n - 1)]
    terms += [(x_coeff, 1 << i, 0) for i in range(n)]
    return terms


def random_pauli_sum(n: int, n_terms: int, seed: int) -> List[Tuple[float, int, int]]:
    """Random Pauli strings with coefficients ~ U[-1, 1] (test input)."""
    rng = rng_for(seed)
    out = []
    for _ in range(n_terms):
        x = int(rng.integers(0, 1 << n))
        z = int(rng.integers(0, 1 << n))
        out.append((float(rng.uniform(-1.0, 1.0)), x, z))
    return out


# ------------------------------------------------------------- test inputs ---

def random_unitary(dim: int, rng: np.random.Generator) -> np.ndarray:
    """Haar-random unitary from the QR factorisation of a complex Gaussian matrix."""
    z = (rng.standard_normal((dim, dim)) + 1j * rng.standard_normal((dim, dim))) / np.sqrt(2.0)
    q, r = np.linalg.qr(z)
    d = np.diag(r)
    return q * (d / np.abs(d))


def matrix_params(m: np.ndarray) -> Tuple[float, ...]:
    flat = np.asarray(m, dtype=np.complex128).reshape(-1)
    return tuple(float(v) for pair in zip(flat.real, flat.imag) for v in pair)


def params_matrix(params: Sequence[float], dim: int) -> np.ndarray:
    a = np.asarray(params, dtype=np.float64)
    return (a[0::2] + 1j * a[1::2]).reshape(dim, dim)


def random_mixed_circuit(n: int, n_gates: int, seed: int, ops: Sequence[str] | None = None) -> List[Gate]:
    """Random circuit over every supported op (test input): random qubits,
    angles ~ U[0, 2pi), Haar-random matrices for mat1/mat2."""
    rng = rng_for(seed)
    if ops is None:
        ops = ONE_QUBIT + (TWO_QUBIT if n >= 2 else ())
    out: List[Gate] = []
    for _ in range(n_gates):
        op = ops[int(rng.integers(0, len(ops)))]
        if op in TWO_QUBIT:
            a, b = (int(v) for v in rng.choice(n, size=2, replace=False))
            if op == "mat2":
                out.append(gate(op, a, b, params=matrix_params(random_unitary(4, rng))))
            elif op == "cp":
                out.append(gate(op, a, b, params=(rng.uniform(0, 2 * np.pi),)))
            else:
                out.append(gate(op, a, b))
        else:
            q = int(rng.integers(0, n))
            if op == "mat1":
                out.append(gate(op, q, params=matrix_params(random_unitary(2, rng))))
            elif op in N_ANGLES:
                out.append(gate(op, q, params=rng.uniform(0, 2 * np.pi, size=N_ANGLES[op])))
            else:
                out.append(gate(op, q))
    return out


def random_state(n: int, seed: int) -> np.ndarray:
    """Normalised complex Gaussian state (test input)."""
    rng = rng_for(seed)
    v = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
    return v / np.linalg.norm(v)

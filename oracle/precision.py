"""Reduced-precision projection, emulated in FP64 (no unique correct result).

Test infrastructure (see the package docstring).

A reduced-precision projection has no single right answer, so the oracle
gives (i) the exact FP64 projection (:mod:`oracle.projection`) and (ii) an
*emulated* one: the same Eq. 11 sum with every low-precision operand rounded
the way the device rounds it and all arithmetic in FP64.  A device result is
then checked to lie within an accumulation envelope around (ii), whose size
comes from :func:`project_magnitude` (the same sum with absolute values).

Rounding (round to nearest even, as the IEEE default): FP64 -> FP32, and
FP64 -> FP32 -> BF16 for BF16 (keep the upper 16 bits of the FP32 pattern).

What stays FP64 (the "diagonal split"): terms whose two factors are both
identity or diagonal, and, in a term with exactly one dense factor, the
diagonal of every square (source == destination) block of that factor.  The
rest of the dense factor is rounded, the input segment is rounded after any
diagonal scaling of the other factor is applied, and the intermediate of a
two-sided record, (A X), is rounded to the operand format before the second
product.
"""
from __future__ import annotations

import numpy as np

from . import projection, sectors


def round_fp32(x) -> np.ndarray:
    return np.asarray(x, dtype=np.float64).astype(np.float32).astype(np.float64)


def round_bf16(x) -> np.ndarray:
    f = np.asarray(x, dtype=np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    u = (u + np.uint64(0x7FFF) + lsb) & np.uint64(0xFFFF0000)
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


ROUND = {"fp32": round_fp32, "bf16": round_bf16}


def _kind(p):
    if p is None:
        return "I"
    return "D" if p.ndim == 1 else "M"


def project_emulated(prob, psi, prec: str, coef=None) -> np.ndarray:
    """Eq. 11 with the operands rounded as described in the module docstring."""
    rnd = ROUND[prec]
    coef = prob.coef if coef is None else np.asarray(coef, dtype=np.float64)
    recs, table, n = projection.records(prob)
    psi = np.asarray(psi, dtype=np.float64)
    y = np.zeros(n)
    for k, pin, pout, pa, pb in recs:
        o, dL, dR = table[pin]
        X = psi[o:o + dL * dR].reshape(dL, dR)
        o2, dL2, dR2 = table[pout]
        ka, kb = _kind(pa), _kind(pb)
        c = coef[k]
        if ka != "M" and kb != "M":
            Z = projection._right_t(pb, projection._left(pa, X))
        elif ka == "M" and kb != "M":
            Xs = projection._right_t(pb, X)
            if pin[0] == pout[0]:  # square block: FP64 diagonal + rounded rest
                d = np.diag(pa)
                R = pa - np.diag(d)
                Z = d[:, None] * Xs + rnd(R) @ rnd(Xs)
            else:
                Z = rnd(pa) @ rnd(Xs)
        elif ka != "M" and kb == "M":
            Xs = projection._left(pa, X)
            if pin[1] == pout[1]:
                d = np.diag(pb)
                R = pb - np.diag(d)
                Z = Xs * d[None, :] + rnd(Xs) @ rnd(R).T
            else:
                Z = rnd(Xs) @ rnd(pb).T
        else:
            T = rnd(rnd(pa) @ rnd(X))
            Z = T @ rnd(pb).T
        y[o2:o2 + dL2 * dR2] += (c * Z).reshape(-1)
    return y


def project_magnitude(prob, psi, coef=None) -> np.ndarray:
    """|c| (|A| |X|) |B|^T summed like Eq. 11: the size of the terms each output
    entry accumulates, used to scale rounding envelopes."""
    coef = prob.coef if coef is None else np.asarray(coef, dtype=np.float64)
    recs, table, n = projection.records(prob)
    psi = np.abs(np.asarray(psi, dtype=np.float64))
    y = np.zeros(n)
    for k, pin, pout, pa, pb in recs:
        o, dL, dR = table[pin]
        X = psi[o:o + dL * dR].reshape(dL, dR)
        o2, dL2, dR2 = table[pout]
        pa_ = None if pa is None else np.abs(pa)
        pb_ = None if pb is None else np.abs(pb)
        Z = projection._right_t(pb_, projection._left(pa_, X))
        y[o2:o2 + dL2 * dR2] += (abs(coef[k]) * Z).reshape(-1)
    return y


def max_contraction(prob) -> int:
    """Longest inner dimension any output entry accumulates over (sum over its
    records of the contraction lengths), for envelope sizing."""
    recs, table, n = projection.records(prob)
    acc = {}
    for k, pin, pout, pa, pb in recs:
        _, di, dk = table[pin]
        ln = (di if (pa is not None and pa.ndim == 2) else 1) + (dk if (pb is not None and pb.ndim == 2) else 1)
        acc[pout] = acc.get(pout, 0) + ln
    return max(acc.values()) if acc else 0


__all__ = ["round_fp32", "round_bf16", "project_emulated", "project_magnitude",
           "max_contraction", "sectors"]

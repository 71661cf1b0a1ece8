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


UNIT = {"fp32": 2.0 ** -24, "bf16": 2.0 ** -8}


def project_envelope(prob, psi, prec: str, coef=None) -> np.ndarray:
    """Elementwise bound on |device - project_emulated| for one output entry.

    The emulation rounds exactly the operands the device rounds, so what is
    left are the device's FP32 sums and, for a record with two dense factors,
    the rounding of its intermediate.  Per record, with mag_rec = |c| |A| |X| |B|^T
    (this record's share of :func:`project_magnitude`):

    * every FP32 sum of length K (FP32/BF16 MFMA accumulate in FP32) is off by
      at most (K + 2) 2^-24 of the sum of its absolute terms (standard
      floating-point summation bound, two guard terms for the product rounding
      inside the matrix instruction);
    * the intermediate of a two-sided record is rounded to the operand format
      (unit u_T); the device may form it as (A X) or as (X B^T), whichever is
      cheaper, while the emulation always forms (A X): both are within
      u_T mag_rec of the product of the rounded operands, hence 2 u_T;
    * the per-record sums, coefficients and diagonal terms are FP64 (their
      errors are ~1e-16 relative and covered by the safety factor).

    The bound is sum_rec gamma_rec mag_rec with gamma = (K_A + K_B + 4) 2^-24
    + 2 u_T [two-sided], times 1.25 for the (1 + u)^3 growth of the rounded
    operands' magnitudes over the unrounded ones used in mag_rec.
    """
    coef = prob.coef if coef is None else np.asarray(coef, dtype=np.float64)
    recs, table, n = projection.records(prob)
    psi = np.abs(np.asarray(psi, dtype=np.float64))
    u32, uT = 2.0 ** -24, UNIT[prec]
    env = np.zeros(n)
    for k, pin, pout, pa, pb in recs:
        o, dL, dR = table[pin]
        X = psi[o:o + dL * dR].reshape(dL, dR)
        o2, dL2, dR2 = table[pout]
        da = pa is not None and pa.ndim == 2
        db = pb is not None and pb.ndim == 2
        if not da and not db:
            continue  # FP64 diagonal term
        pa_ = None if pa is None else np.abs(pa)
        pb_ = None if pb is None else np.abs(pb)
        mag = abs(coef[k]) * projection._right_t(pb_, projection._left(pa_, X))
        gamma = ((dL if da else 0) + (dR if db else 0) + (4 if da and db else 2)) * u32
        if da and db:
            gamma += 2.0 * uT
        env[o2:o2 + dL2 * dR2] += gamma * mag.reshape(-1)
    return 1.25 * env


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


__all__ = ["round_fp32", "round_bf16", "project_emulated", "project_magnitude", "project_envelope",
           "max_contraction", "sectors"]

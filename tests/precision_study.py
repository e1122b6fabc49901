"""Precision study of the DFT-GEMM formulation of Q_h (section 3.3): CPU
emulations of the GPU dataflow under different arithmetic, each compared
with the FP64 oracle by the batch relative L2 error (and the worst cell).

This is a study script beside the tests, not a test and not the oracle: it
emulates number formats with NumPy (FP16 and FP32 roundings, FP32 matrix
products as the accumulation of the matrix cores) on the oracle's filters,
and it shares nothing with the HIP library. It reproduces the precision
tables that motivate the mixed path's design:

  2D (hard spheres, 32x32 on [-8,8]^2, M = 8, the packed transforms):
    fp32_mfma     DFT-GEMMs in FP32 with FP32 spectra, filters and fields
    fp16x3_f32    FP16 hi + lo operands, three products, FP32 accumulation,
                  power-of-two range scaling per pass, FP32 intermediates
    exact_f32     exact GEMMs, every intermediate rounded to FP32
    fx16_f32filt  the fixed-point-lead split (lead on the integer grid + FP16
                  hi and lo, six products), FP64 intermediates, FP32 filters
    fx16          the same with FP64 filters (the mixed path as built)
    fx16_no_lo_data, fx16_no_lo_dft
                  fx16 without the product (data lo) x (DFT lead), or without
                  (data lead) x (DFT lo): five products each

  3D (hard spheres, M = 8): the FP32-intermediate FX16 variant, and which of
  its FP32 roundings (spectrum, filters, filter products, the three inverse
  passes, the loss transform) set its error.

    python tests/precision_study.py [--cells 64] [--only 2d|3d]
"""

from __future__ import annotations

import argparse
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import workloads as wl  # noqa: E402
from oracle import spectral as sp  # noqa: E402

F32, F16 = np.float32, np.float16


def r32(x):
    """Round to FP32 (complex parts separately), back in FP64."""
    if np.iscomplexobj(x):
        return x.real.astype(F32).astype(np.float64) + 1j * x.imag.astype(F32).astype(np.float64)
    return x.astype(F32).astype(np.float64)


def pow2_scale(x, top: int) -> float:
    """Power of two that brings max |x| below 2^top."""
    m = float(np.max(np.abs(x))) if x.size else 0.0
    if m == 0.0:
        return 1.0
    return 2.0 ** (top - np.frexp(m)[1])


# ----------------------------------------------------------- GEMM arithmetic
# A complex pass Y = X E over the last axis is one real GEMM with K = 2N:
# [Xr | Xi] @ [[Er, Ei], [-Ei, Er]], as the kernels lay it out.

def _real_operands(X, E):
    A = np.concatenate([X.real, X.imag], axis=-1)
    B = np.block([[E.real, E.imag], [-E.imag, E.real]])
    return A, B


def _finish(Y, n):
    return Y[..., :n] + 1j * Y[..., n:]


def gemm_exact(X, E):
    return X @ E


def gemm_fp32(X, E):
    A, B = _real_operands(X, E)
    return _finish((A.astype(F32) @ B.astype(F32)).astype(np.float64), E.shape[1])


def _split3(y):
    """Lead on the integer grid, FP16 hi and lo of the remainder (|y| < 2^9)."""
    lead = np.rint(y)
    r = (y - lead).astype(F32)
    hi = r.astype(F16).astype(F32)
    lo = (r - hi).astype(F16).astype(F32)
    return lead.astype(F32), hi, lo


def gemm_fx16(X, E, lo_data: bool = True, lo_dft: bool = True):
    """Six FP16 products with FP32 accumulation: lead x lead exact in one
    accumulator, the five corrections in a second; returns the FP64 sum.
    lo_data / lo_dft = False leave out (data lo) x (DFT lead) / (data lead) x
    (DFT lo)."""
    A, B = _real_operands(X, E)
    sa, sb = pow2_scale(A, 9), 512.0
    al, ah, ao = _split3(A * sa)
    bl, bh, bo = _split3(B * sb)
    acc0 = (al.astype(np.float64) @ bl.astype(np.float64)).astype(F32)    # exact integer sums < 2^24
    zero = np.zeros((A.shape[0], B.shape[1]), dtype=F32)
    acc1 = (al @ bh + ah @ bl + (al @ bo if lo_dft else zero) + ah @ bh       # FP32 accumulation
            + (ao @ bl if lo_data else zero))
    Y = (acc0.astype(np.float64) + acc1.astype(np.float64)) / (sa * sb)
    return _finish(Y, E.shape[1])


def gemm_fp16x3(X, E):
    """FP16 hi + lo operands, three products (hi hi + hi lo + lo hi) with FP32
    accumulation and a power-of-two range scale; FP32 result."""
    A, B = _real_operands(X, E)
    sa, sb = pow2_scale(A, 14), 2.0 ** 14
    ah = (A * sa).astype(F16).astype(F32)
    al = ((A * sa).astype(F32) - ah).astype(F16).astype(F32)
    bh = (B * sb).astype(F16).astype(F32)
    bl = ((B * sb).astype(F32) - bh).astype(F16).astype(F32)
    acc = ah @ bh + ah @ bl + al @ bh
    return _finish(acc.astype(np.float64) / (sa * sb), E.shape[1])


# ------------------------------------------------------------- 2D pipeline

def dft_mats(N):
    j = np.arange(N)
    ang = 2.0 * np.pi * np.outer(j, j) / N
    return np.exp(-1j * ang), np.exp(1j * ang)


def packed_filters_2d(s: sp.Setup):
    """Packed complex filters of the 2D plans: direction p and its
    perpendicular p + M/2 share one inverse transform, m = sqrt|2W| (sign(W)
    alpha_p + i alpha_{p+M/2}), so that Re * Im of its inverse DFT is the
    pair's gain 2 W g_p g_{p+M/2}; the loss multiplier separately."""
    bank = sp.filter_bank(s)
    K = len(bank) // s.M
    out = []
    for p in range(s.M // 2):
        for j in range(K):
            W, a, _ = bank[p * K + j]
            _, b, _ = bank[(p + s.M // 2) * K + j]
            out.append(np.sqrt(abs(2 * W)) * (np.sign(W) * a + 1j * b))
    return out, sp.loss_multiplier(bank)


def q_2d(f, mats, packed, loss, gemm, inter, filt):
    """Q of one N x N cell by DFT-GEMM passes. gemm: pass arithmetic; inter:
    rounding of every intermediate (spectrum, filter products, the field
    between the two inverse passes, the fields); filt: rounding of the filters."""
    Ef, Ei = mats
    n2 = f.shape[0] ** 2
    x = inter(gemm(f.astype(np.complex128), Ef))          # along axis 1
    fh = inter(gemm(x.T, Ef))                             # along axis 0 (transposed layout)
    gain = np.zeros(f.shape)
    for m in packed:
        z = inter(filt(m.T) * fh)
        y = inter(gemm(inter(gemm(z, Ei)).T, Ei)) / n2
        gain += y.real * y.imag
    z = inter(filt(loss.T) * fh)
    L = inter(gemm(inter(gemm(z, Ei)).T, Ei)).real / n2
    return gain - f * L


def study_2d(cells: int, seed: int = 1001):
    N, L, M = 32, 8.0, 8
    s = sp.Setup(d=2, N=N, L=L, kernel="hard_sphere", M=M)
    f = wl.mixture_cells(2, N, L, cells, seed).astype(F32).astype(np.float64)
    ref = sp.q_fast(f, s)
    mats = dft_mats(N)
    packed, loss = packed_filters_2d(s)
    ident = lambda x: x   # noqa: E731
    variants = {
        "fp32_mfma": (gemm_fp32, r32, r32),
        "fp16x3_f32": (gemm_fp16x3, r32, r32),
        "exact_f32": (gemm_exact, r32, r32),
        "fx16_f32filt": (gemm_fx16, ident, r32),
        "fx16": (gemm_fx16, ident, ident),
        "fx16_no_lo_data": (lambda X, E: gemm_fx16(X, E, lo_data=False), ident, ident),
        "fx16_no_lo_dft": (lambda X, E: gemm_fx16(X, E, lo_dft=False), ident, ident),
    }
    out = {}
    for name, (g, inter, filt) in variants.items():
        q = np.stack([q_2d(f[c], mats, packed, loss, g, inter, filt) for c in range(cells)])
        out[name] = metrics(q, ref)
    out["packing_exact"] = metrics(np.stack([q_2d(f[c], mats, packed, loss, gemm_exact, ident, ident)
                                             for c in range(cells)]), ref)
    return out


# ------------------------------------------------------------- 3D pipeline

def _passes3(x, inv, rnd):
    axes = (0, 1, 2) if inv else (2, 1, 0)
    for i, ax in enumerate(axes):
        x = np.fft.ifft(x, axis=ax) * x.shape[ax] if inv else np.fft.fft(x, axis=ax)
        if rnd[i]:
            x = r32(x)
    return x


def q_3d(f, s, bank, fwd, filt, z32, inv, linv, lfilt):
    """Q of one 3D cell with exact passes and FP32 roundings where flagged:
    fwd/inv/linv per pass (forward; gain and loss inverse), filt/lfilt the
    stored filters, z32 the filter products."""
    n3 = s.N ** 3
    fh = _passes3(f.astype(np.complex128), False, fwd)
    gain = np.zeros_like(f)
    for W, a, ap in bank:
        m = np.sqrt(abs(W)) * (np.sign(W) * a + 1j * ap) / n3
        z = (r32(m) if filt else m) * fh
        y = _passes3(r32(z) if z32 else z, True, inv)
        gain += y.real * y.imag
    lm = sp.loss_multiplier(bank) / n3
    z = (r32(lm) if lfilt else lm) * fh
    y = _passes3(r32(z) if z32 else z, True, linv)
    return gain - f * y.real


def study_3d(cells: int, grids=(16, 20, 32)):
    T, F = True, False
    base = dict(fwd=(F, F, F), filt=F, z32=F, inv=(F, F, F), linv=(F, F, F), lfilt=F)
    allr = dict(fwd=(T, T, T), filt=T, z32=T, inv=(T, T, T), linv=(T, T, T), lfilt=T)
    out = {}
    for N in grids:
        s = sp.Setup(d=3, N=N, L=8.0, kernel="hard_sphere", M=8)
        bank = sp.filter_bank(s)
        f = wl.mixture_cells(3, N, 8.0, cells, 40 + N).astype(F32).astype(np.float64)
        ref = np.stack([sp.q_fast(f[c], s, bank) for c in range(cells)])
        row = {}
        for name, kw in [("fp32_intermediates", allr)] + [
                (f"only_{k}", dict(base, **{k: allr[k]})) for k in base]:
            q = np.stack([q_3d(f[c], s, bank, **kw) for c in range(cells)])
            row[name] = metrics(q, ref)
        out[N] = row
    return out


def metrics(q, ref):
    n = q.shape[0]
    err = float(np.linalg.norm(q - ref) / np.linalg.norm(ref))
    cell = float((np.linalg.norm((q - ref).reshape(n, -1), axis=1)
                  / np.linalg.norm(ref.reshape(n, -1), axis=1)).max())
    return err, cell


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--cells", type=int, default=64)
    ap.add_argument("--cells3d", type=int, default=8)
    ap.add_argument("--only", choices=["2d", "3d"])
    args = ap.parse_args()
    if args.only != "3d":
        print(f"2D hard spheres 32x32, M=8, {args.cells} cells (hs2d_32 inputs): rel L2 / worst cell")
        for k, (e, c) in study_2d(args.cells).items():
            print(f"  {k:14s} {e:.2e}  {c:.2e}", flush=True)
    if args.only != "2d":
        print(f"3D hard spheres, M=8, {args.cells3d} cells per grid: rel L2 / worst cell")
        for N, row in study_3d(args.cells3d).items():
            for k, (e, c) in row.items():
                print(f"  N={N:2d} {k:22s} {e:.2e}  {c:.2e}", flush=True)


if __name__ == "__main__":
    main()

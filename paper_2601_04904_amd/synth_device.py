"""Seeded synthetic inputs generated directly in device memory (torch on ROCm).

Same recipe as synth.py (see its header), drawn with a seeded torch.Generator
on the device so that large serving requests (blocks up to 1024, n up to 256,
many GB per matrix) need neither host generation nor a PCIe upload.  The
values are not bit-identical to synth.py's NumPy stream; this generator is
used where only the structure matters (timing, serving), and parity tests
use synth.py.  No arithmetic of the method is done here.

The blocks are written into given DeviceBlocks (or new ones) a few at a time,
so the temporaries stay small whatever the request's size.
"""
from __future__ import annotations

import math

CHUNK = 8      # blocks generated at once


def _cn(torch, g, shape, var, device):
    # complex normal with E|z|^2 = var (re and im each var/2)
    z = torch.randn(shape, dtype=torch.complex128, generator=g, device=device)
    return z * math.sqrt(var)


def _hermitian(torch, g, m, count, device):
    M = _cn(torch, g, (count, m, m), 1.0, device)
    H = (M + M.conj().transpose(-1, -2)) / math.sqrt(2.0 * m)
    onsite = torch.rand((count, m), dtype=torch.float64, generator=g, device=device) * 2.0 - 1.0
    return H + torch.diag_embed(onsite.to(torch.complex128))


def _chunks(count):
    for s in range(0, count, CHUNK):
        yield s, min(count, s + CHUNK)


def _empty(n, b, a, device):
    from .solver import DeviceBlocks
    return DeviceBlocks.empty(n, b, a, device=device)


def gen_A_device(n, b, a=0, E=0.3, eta=1e-3, seed=0, device="cuda", out=None):
    """A (DeviceBlocks) built on the device, into `out` if given."""
    import torch
    A = out if out is not None else _empty(n, b, a, device)
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    z = complex(E, eta)
    eye = torch.eye(b, dtype=torch.complex128, device=device)
    for s, e in _chunks(n):
        A.diag[s:e] = z * eye - _hermitian(torch, g, b, e - s, device)
    A.diag[0] += 0.5j * eye
    if n > 1:
        A.diag[n - 1] += 0.5j * eye
    for s, e in _chunks(max(n - 1, 0)):
        T = _cn(torch, g, (e - s, b, b), 0.5 / b, device)
        A.upper[s:e] = -T
        A.lower[s:e] = -T.conj().transpose(-1, -2)
    if a > 0:
        for s, e in _chunks(n):
            K = _cn(torch, g, (e - s, b, a), 0.1 / b, device)
            A.arrow_right[s:e] = -K
            A.arrow_bottom[s:e] = -K.conj().transpose(-1, -2)
        eyea = torch.eye(a, dtype=torch.complex128, device=device)
        A.tip[:] = z * eyea - _hermitian(torch, g, a, 1, device)[0] + 0.5j * eyea
    return A


def gen_rhs_device(n, b, a=0, seed=0, device="cuda", out=None):
    """An anti-Hermitian right-hand side B = Sigma^< on the same pattern."""
    import torch
    B = out if out is not None else _empty(n, b, a, device)
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    for s, e in _chunks(n):
        C = _cn(torch, g, (e - s, b, b), 1.0, device)
        B.diag[s:e] = 1j * torch.matmul(C, C.conj().transpose(-1, -2).contiguous()) / b
    for s, e in _chunks(max(n - 1, 0)):
        D = _cn(torch, g, (e - s, b, b), 1.0, device)
        B.upper[s:e] = 0.1j * D
        B.lower[s:e] = 0.1j * D.conj().transpose(-1, -2)
    if a > 0:
        for s, e in _chunks(n):
            F = _cn(torch, g, (e - s, b, a), 1.0, device)
            B.arrow_right[s:e] = 0.1j * F
            B.arrow_bottom[s:e] = 0.1j * F.conj().transpose(-1, -2)
        Ct = _cn(torch, g, (a, a), 1.0, device)
        B.tip[:] = 1j * (Ct @ Ct.conj().T.contiguous()) / a
    return B


def gen_problem_device(n, b, a=0, E=0.3, eta=1e-3, seed=0, device="cuda", with_B=True, out=None):
    """(A, B) as DeviceBlocks built on the device (into out = (A, B) if given)."""
    oA, oB = out if out is not None else (None, None)
    A = gen_A_device(n, b, a, E, eta, seed, device, oA)
    if not with_B:
        return A, None
    return A, gen_rhs_device(n, b, a, seed + 7919, device, oB)

"""Seeded synthetic inputs generated directly in device memory (torch on ROCm).

Same recipe as synth.py (see its header), drawn with a seeded torch.Generator
on the device so that large serving requests (blocks up to 1024, n up to 256,
many GB per matrix) need neither host generation nor a PCIe upload.  The
values are not bit-identical to synth.py's NumPy stream; this generator is
used where only the structure matters (timing, serving), and parity tests
use synth.py.  No arithmetic of the method is done here.
"""
from __future__ import annotations

import math


def _cn(torch, g, shape, var, device):
    # complex normal with E|z|^2 = var (re and im each var/2)
    z = torch.randn(shape, dtype=torch.complex128, generator=g, device=device)
    return z * math.sqrt(var)


def _hermitian(torch, g, m, count, device):
    M = _cn(torch, g, (count, m, m), 1.0, device)
    H = (M + M.conj().transpose(-1, -2)) / math.sqrt(2.0 * m)
    onsite = torch.rand((count, m), dtype=torch.float64, generator=g, device=device) * 2.0 - 1.0
    return H + torch.diag_embed(onsite.to(torch.complex128))


def gen_problem_device(n, b, a=0, E=0.3, eta=1e-3, seed=0, device="cuda", with_B=True):
    """(A, B) as DeviceBlocks built on the device."""
    import torch
    from .solver import DeviceBlocks
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    z = complex(E, eta)
    eye = torch.eye(b, dtype=torch.complex128, device=device)
    diag = z * eye - _hermitian(torch, g, b, n, device)
    diag[0] += 0.5j * eye
    if n > 1:
        diag[n - 1] += 0.5j * eye
    T = _cn(torch, g, (max(n - 1, 0), b, b), 0.5 / b, device)
    upper = (-T).contiguous()
    lower = (-T.conj().transpose(-1, -2)).contiguous()
    if a > 0:
        K = _cn(torch, g, (n, b, a), 0.1 / b, device)
        ar = (-K).contiguous()
        ab = (-K.conj().transpose(-1, -2)).contiguous()
        eyea = torch.eye(a, dtype=torch.complex128, device=device)
        tip = (z * eyea - _hermitian(torch, g, a, 1, device)[0] + 0.5j * eyea).contiguous()
    else:
        ar = torch.empty((n, b, 0), dtype=torch.complex128, device=device)
        ab = torch.empty((n, 0, b), dtype=torch.complex128, device=device)
        tip = torch.empty((0, 0), dtype=torch.complex128, device=device)
    A = DeviceBlocks(diag.contiguous(), upper, lower, ar, ab, tip)
    if not with_B:
        return A, None
    return A, gen_rhs_device(n, b, a, seed + 7919, device)


def gen_rhs_device(n, b, a=0, seed=0, device="cuda"):
    """An anti-Hermitian right-hand side B = Sigma^< on the same pattern."""
    import torch
    from .solver import DeviceBlocks
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    C = _cn(torch, g, (n, b, b), 1.0, device)
    diag = 1j * torch.matmul(C, C.conj().transpose(-1, -2).contiguous()) / b
    D = _cn(torch, g, (max(n - 1, 0), b, b), 1.0, device)
    upper = (0.1j * D).contiguous()
    lower = (0.1j * D.conj().transpose(-1, -2)).contiguous()
    if a > 0:
        F = _cn(torch, g, (n, b, a), 1.0, device)
        ar = (0.1j * F).contiguous()
        ab = (0.1j * F.conj().transpose(-1, -2)).contiguous()
        Ct = _cn(torch, g, (a, a), 1.0, device)
        tip = (1j * (Ct @ Ct.conj().T.contiguous()) / a).contiguous()
    else:
        ar = torch.empty((n, b, 0), dtype=torch.complex128, device=device)
        ab = torch.empty((n, 0, b), dtype=torch.complex128, device=device)
        tip = torch.empty((0, 0), dtype=torch.complex128, device=device)
    return DeviceBlocks(diag.contiguous(), upper, lower, ar, ab, tip)

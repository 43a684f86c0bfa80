"""Seeded input generators that run on the GPU, for inputs too large to draw quickly on the host.

They hold none of the sort's arithmetic.  A test that needs the oracle copies the generated
bytes back to the host first, so both sides see exactly the same input.
"""
import torch


def _gen(seed: int, device) -> torch.Generator:
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    return g


def u64_uniform(n: int, seed: int, device="cuda:0") -> torch.Tensor:
    """n keys uniform over the 64-bit range, returned as an int64 tensor holding the uint64 bits."""
    return torch.randint(-(2**63), 2**63 - 1, (n,), dtype=torch.int64, device=device, generator=_gen(seed, device))


def zipf_u64(n: int, seed: int, s: float = 1.1, vmax: int = 2**32, device="cuda:0",
             chunk: int = 1 << 26) -> torch.Tensor:
    """Zipf(s) ranks on {1..vmax} by rejection-inversion (Hormann and Derflinger, 1996), as an
    int64 tensor holding the uint64 bits.  H is the integral of x^-s, Hinv its inverse."""
    g = _gen(seed, device)
    q = 1.0 - s

    def H(x):
        return torch.expm1(q * torch.log(x)) / q

    def Hinv(y):
        return torch.exp(torch.log1p(q * y) / q)

    def h(x):
        return torch.exp(-s * torch.log(x))

    t = lambda v: torch.tensor(v, dtype=torch.float64, device=device)
    hx1 = float(H(t(1.5))) - 1.0
    hn = float(H(t(vmax + 0.5)))
    squeeze = 2.0 - float(Hinv(H(t(2.5)) - h(t(2.0))))
    out = torch.empty(n, dtype=torch.int64, device=device)
    for c0 in range(0, n, chunk):
        m = min(chunk, n - c0)
        todo = torch.arange(c0, c0 + m, device=device)
        while todo.numel():
            u = hn + torch.rand(todo.numel(), dtype=torch.float64, device=device, generator=g) * (hx1 - hn)
            x = Hinv(u)
            k = torch.clamp(torch.floor(x + 0.5), 1.0, float(vmax))
            ok = (k - x <= squeeze) | (u >= H(k + 0.5) - h(k))
            out[todo[ok]] = k[ok].to(torch.int64)
            todo = todo[~ok]
    return out

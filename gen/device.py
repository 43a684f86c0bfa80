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


# ---------------------------------------------------------------- fp64 distributions on the device
# The same recipes as the host generators (different random streams): normal(0,1),
# lognormal(0, sigma), exponential(lam), a mixture of m N(mu_i, 1) with mu_i ~ U[-100, 100] and
# equal weights, integers uniform in [0, hi) as fp64, and U[0, 1).
DEVICE_DISTS = ("uniform01", "normal", "lognormal", "exponential", "mixgauss", "uniform_int", "lognormal2",
                "mixgauss20")


def fp64(dist: str, n: int, seed: int, device="cuda:0", out: torch.Tensor | None = None) -> torch.Tensor:
    """n fp64 keys of a named distribution, written into `out` when given."""
    g = _gen(seed, device)
    x = out if out is not None else torch.empty(n, dtype=torch.float64, device=device)
    if dist == "uniform01":
        x.uniform_(0.0, 1.0, generator=g)
    elif dist == "normal":
        x.normal_(0.0, 1.0, generator=g)
    elif dist in ("lognormal", "lognormal2"):
        x.log_normal_(0.0, 0.5 if dist == "lognormal" else 2.0, generator=g)
    elif dist == "exponential":
        x.exponential_(2.0, generator=g)
    elif dist in ("mixgauss", "mixgauss20"):
        m = 5 if dist == "mixgauss" else 20
        means = torch.empty(m, dtype=torch.float64, device=device).uniform_(-100.0, 100.0, generator=g)
        comp = torch.randint(0, m, (n,), device=device, generator=g)
        x.normal_(0.0, 1.0, generator=g)
        x.add_(means[comp])
    elif dist == "uniform_int":
        x.copy_(torch.randint(0, 1_000_000, (n,), device=device, generator=g))
    else:
        raise ValueError(dist)
    return x


def request_keys(dist: str, n: int, seed: int, dtype: int, out: torch.Tensor, device="cuda:0") -> None:
    """A served request's keys into `out`: fp64 as drawn, uint64 = floor(|x| * 2^32) (written as
    int64 bits), fp32 = x rounded to nearest."""
    if dtype == 0:
        fp64(dist, n, seed, device, out=out)
        return
    x = fp64(dist, n, seed, device)
    if dtype == 1:
        out.copy_(x)
    else:
        y = torch.floor(torch.abs(x) * 4294967296.0)
        # values reach 2^64 only for |x| >= 2^32, which these distributions do not draw
        big = y >= 9223372036854775808.0
        lo = torch.where(big, y - 18446744073709551616.0, y).to(torch.int64)
        out.view(torch.int64).copy_(lo)

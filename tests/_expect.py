"""Expected values computed in the tests themselves (no product code)."""
import math


def rounded_gaussian_pmf(sigma: float, lo: int, hi: int):
    """P(sat(round(N(0, sigma^2))) = v) for v in [lo, hi] (exact, via erf)."""
    def cdf(z):
        return 0.5 * (1.0 + math.erf(z / (sigma * math.sqrt(2.0))))
    pmf = []
    for v in range(lo, hi + 1):
        a = -math.inf if v == lo else v - 0.5
        b = math.inf if v == hi else v + 0.5
        pa = 0.0 if a == -math.inf else cdf(a)
        pb = 1.0 if b == math.inf else cdf(b)
        pmf.append(pb - pa)
    return pmf

"""The one-dimensional convergence study of Section 4 on the GPU.

Domain [-pi, pi] as the periodic grid of N = 2^n points (l = 2 pi, the grid
x_i = i pi / 2^(n-1)); covariance with the spectral density of Section 4,
which in the cycles convention is the Matern density with nu = 7/2 and
ell = sqrt(0.07), so that the closed form is
    C(x) = (200/3 |x|^3 + 40 x^2 + 10 |x| + 1) exp(-10 |x|).
For each n the statistical covariance (1/S) sum_j eta_j(0) eta_j(x_i) over S
samples (grf_covariance: the fields are generated and accumulated on the GPU,
never stored) is compared with C on every grid point; e_n is the largest
difference.  The paper reports an order of at least N^-4 until the Monte Carlo
error (about sqrt(2 / S)) takes over.

    python -m paper_1105_2737_amd.study [--samples 100000000] [--nmin 2] [--nmax 12]

prints one JSON line per grid and a summary line.
"""
import argparse
import json
import math
import time


def closed_form(x):
    ax = abs(x)
    return (200.0 / 3.0 * ax ** 3 + 40.0 * ax ** 2 + 10.0 * ax + 1.0) * math.exp(-10.0 * ax)


def run(samples=10 ** 8, nmin=2, nmax=12, seed=0, dtype="float32", out=print):
    import torch

    from . import Plan
    l = 2.0 * math.pi
    dt = torch.float32 if dtype == "float32" else torch.float64
    rows = []
    for n in range(nmin, nmax + 1):
        N = 2 ** n
        plan = Plan((N,), lengths=(l,), alg=2, dtype=dt, cov="matern", sigma=1.0,
                    length_scale=math.sqrt(0.07), nu=3.5)
        plan.covariance(seed=seed, nsamples=min(samples, 1024))      # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        cov = plan.covariance(seed=seed, nsamples=samples)
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        c = cov.cpu().tolist()
        err = max(abs(c[j] - closed_form(min(j, N - j) * l / N)) for j in range(N))
        row = {"n": n, "N": N, "samples": samples, "e_n": err, "e_n_times_N4": err * N ** 4,
               "seconds": round(sec, 4), "points_per_s": round(samples * N / sec, 1)}
        rows.append(row)
        out(json.dumps(row))
    slopes = [math.log2(rows[i + 1]["e_n"] / rows[i]["e_n"]) for i in range(len(rows) - 1)]
    summary = {"slopes_per_doubling": [round(s, 3) for s in slopes],
               "monte_carlo_error_scale": math.sqrt(2.0 / samples), "dtype": dtype}
    out(json.dumps(summary))
    return rows, summary


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--samples", type=int, default=10 ** 8)
    ap.add_argument("--nmin", type=int, default=2)
    ap.add_argument("--nmax", type=int, default=12)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--dtype", choices=("float32", "float64"), default="float32")
    a = ap.parse_args()
    run(a.samples, a.nmin, a.nmax, a.seed, a.dtype, out=lambda s: print(s, flush=True))


if __name__ == "__main__":
    main()

"""Write the stored expected values used by the tests and the benchmark.

Every number written here comes from the FP64 oracle (oracle/sb2_oracle.py)
applied to the seeded synthetic inputs of paper_1905_01180_amd.inputs; nothing
comes from the HIP library.  Run from the repository root:

    python tests/golden/make_golden.py --config 0        # N=10,  T=20   (seconds)
    python tests/golden/make_golden.py --config 1        # N=50,  T=500  (minutes)
    python tests/golden/make_golden.py --config 2        # N=100, T=1000 (hours; resumable)

Output: tests/golden/oracle_c<id>.npz with
    i_ns         (N, N) complex128  collision integral I_ns(t), t = T dt
    sigma_ks     (K,)   int64       past-time indices whose self-energies are stored
    sigma_less   (K, N, N)          Sigma^<(t, t_k) for k in sigma_ks
    sigma_great  (K, N, N)          Sigma^>(t, t_k)
    term_norms   (T,)   float64     Frobenius norm of dt [Sigma^> G^<(t_k,t) - Sigma^< G^>(t_k,t)]
Per-past-time partial results are checkpointed under tests/golden/.partial_c<id>/
so that a long run can be resumed.
"""
import argparse
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import sb2_oracle as o  # noqa: E402
from paper_1905_01180_amd import inputs as gen  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def sampled_ks(t_len):
    if t_len <= 32:
        return list(range(t_len))
    ks = sorted({0, 1, t_len // 2, t_len - 2, t_len - 1})
    return [k for k in ks if 0 <= k < t_len]


def run(config_id: int, every: int = 1):
    s = gen.make_config(config_id)
    t_len, n = s.t, s.n
    part = os.path.join(HERE, f".partial_c{config_id}")
    os.makedirs(part, exist_ok=True)
    keep = set(sampled_ks(t_len))
    w = o.exchange_combined(s.v)
    zero = np.zeros((n, n), np.complex128)
    t0 = time.time()
    for k in range(t_len):
        f = os.path.join(part, f"k{k:05d}.npz")
        if os.path.exists(f):
            continue
        u = o.propagator(s.h, (t_len - k) * s.dt)
        gl, gg, gl_bar, gg_bar = o.gkba_pair(u, s.rho_hist[k], zero)
        s_less = o.sigma(s.v, gl, gg_bar, w)
        s_great = o.sigma(s.v, gg, gl_bar, w)
        term = s_great @ gl_bar - s_less @ gg_bar
        extra = dict(s_less=s_less, s_great=s_great) if k in keep else {}
        np.savez(f + ".tmp.npz", term=term, **extra)
        os.replace(f + ".tmp.npz", f)
        if k % every == 0:
            print(f"c{config_id} k={k}/{t_len} {time.time() - t0:.0f}s", flush=True)
    acc = np.zeros((n, n), np.complex128)
    norms = np.zeros(t_len)
    sl, sg = [], []
    for k in range(t_len):                       # k-ordered FP64 sum, as the oracle's collision()
        z = np.load(os.path.join(part, f"k{k:05d}.npz"))
        acc += z["term"]
        norms[k] = s.dt * np.linalg.norm(z["term"])
        if k in keep:
            sl.append(z["s_less"])
            sg.append(z["s_great"])
    i_ns = s.dt * acc
    out = os.path.join(HERE, f"oracle_c{config_id}.npz")
    np.savez(out, i_ns=i_ns, sigma_ks=np.array(sorted(keep), np.int64), sigma_less=np.stack(sl),
             sigma_great=np.stack(sg), term_norms=norms, n=n, t=t_len, dt=s.dt)
    print("wrote", out)


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--config", type=int, required=True, choices=[0, 1, 2, 3])
    ap.add_argument("--every", type=int, default=10)
    a = ap.parse_args()
    run(a.config, a.every)

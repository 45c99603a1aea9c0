"""Write synth/manifest.json: kappa_c of every synthetic gauge field used by
the workloads (the operator of Example 7 runs at kappa near kappa_critical).

Calls only the oracle and the seeded generators. kappa_c = 1 / max Re
lambda(D) from a dense eigensolve (n <= 3072) or ARPACK, cross-checked by
bisection on the positivity predicate.

usage: python -m oracle.make_manifest C1 C2 ...   (default: C1 C2 C3)
"""
import json
import sys
import time

import numpy as np

import synth
from oracle import kappa


def compute(name):
    cfg = synth.CONFIGS[name]
    dims = cfg["dims"]
    t0 = time.time()
    links = synth.gauge_links(dims, cfg["eps"], cfg["seed"])
    n = 12 * int(np.prod(dims))
    if n <= 3072:
        ev = kappa.rightmost_dense(links)
        method = "dense eig"
    elif n <= 100000:
        ev = kappa.rightmost_arpack(links)
        method = "arpack LR nev=6 ncv=64 tol=1e-8"
    else:
        # large lattices: the spectral edge is dense and ARPACK does not
        # converge in hours on a few cores; a restarted Arnoldi estimate of the
        # rightmost eigenvalue (Ritz residual recorded) is used instead --
        # kappa = 0.98 kappa_c needs kappa_c only to far better than 2 %
        m, restarts = (60, 8) if n <= 10_000_000 else (40, 6)
        ev, res = kappa.rightmost_restarted_arnoldi(links, m=m, restarts=restarts)
        method = "restarted Arnoldi m=%d, %d restarts, Ritz residual %.2e" % (m, restarts, res)
    kc = kappa.kappa_c_from_eigs(ev)
    kb = kappa.bisect_kappa_c(ev)
    if abs(kb - kc) > 1e-9 * kc:
        raise RuntimeError("bisection disagrees: %r vs %r" % (kb, kc))
    top = ev[np.argsort(-ev.real)][:6]
    return dict(dims=list(dims), eps=cfg["eps"], seed=cfg["seed"],
                lambda_R=float(np.max(ev.real)), kappa_c=kc,
                kappa_c_bisect=kb, method=method,
                rightmost=[[float(z.real), float(z.imag)] for z in top],
                seconds=round(time.time() - t0, 1))


def main(names):
    for name in names:
        cfg = synth.CONFIGS[name]
        key = synth.manifest_key(cfg["dims"], cfg["eps"], cfg["seed"])
        entry = compute(name)
        data = synth.manifest()          # re-read: other runs may have added keys
        data[key] = entry
        with open(synth.MANIFEST, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
        print(name, key, entry["kappa_c"], entry["seconds"], "s", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:] or ["C1", "C2", "C3"])

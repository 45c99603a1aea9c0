"""Lattice indexing for the Wilson-Dirac operator (Example 7's matrix).

The paper does not fix a storage order; this module defines the indexing the
library's tables are checked against bit for bit:

* lex(x,y,z,t) = x + Lx*(y + Ly*(z + Lz*t)), parity p = (x+y+z+t) mod 2,
* even-odd position eo = p*V/2 + (lex >> 1) (one-to-one because Lx is even),
* neighbour table nbr[eo][d] in even-odd positions for the eight hops
  d = +x,+y,+z,+t,-x,-y,-z,-t with periodic wrap,
* sign[eo][d] = -1 when the hop crosses the time boundary (+t from t=Lt-1,
  -t from t=0), else +1. The antiperiodic sign is applied by the operator
  when bc[t] = -1.

Everything here is a plain loop over sites (tiny lattices only for tests that
need the full table; ``tables`` is vectorised and exact).
"""
import numpy as np


def coords(dims):
    """Arrays x, y, z, t of every site in lexicographic order."""
    lx, ly, lz, lt = dims
    lex = np.arange(lx * ly * lz * lt, dtype=np.int64)
    x = lex % lx
    y = (lex // lx) % ly
    z = (lex // (lx * ly)) % lz
    t = lex // (lx * ly * lz)
    return x, y, z, t


def lex_of(dims, x, y, z, t):
    lx, ly, lz, lt = dims
    return x + lx * (y + ly * (z + lz * t))


def eo_of_lex(dims):
    lx, ly, lz, lt = dims
    if any(d % 2 for d in dims):
        raise ValueError("all lattice extents must be even")
    vol = lx * ly * lz * lt
    x, y, z, t = coords(dims)
    p = (x + y + z + t) % 2
    lex = np.arange(vol, dtype=np.int64)
    return (p * (vol // 2) + (lex >> 1)).astype(np.int32)


def tables(dims):
    """(eo_of_lex, nbr, sign): nbr and sign are indexed by even-odd position."""
    lx, ly, lz, lt = dims
    vol = lx * ly * lz * lt
    eo = eo_of_lex(dims)
    x, y, z, t = coords(dims)
    ext = (lx, ly, lz, lt)
    nbr_lex = np.zeros((vol, 8), dtype=np.int64)
    sign_lex = np.ones((vol, 8), dtype=np.int8)
    c = [x, y, z, t]
    for mu in range(4):
        for d, step in ((mu, +1), (mu + 4, -1)):
            cc = [a.copy() for a in c]
            cc[mu] = (c[mu] + step) % ext[mu]
            nbr_lex[:, d] = lex_of(dims, *cc)
            if mu == 3:
                cross = (t == lt - 1) if step > 0 else (t == 0)
                sign_lex[cross, d] = -1
    nbr = np.zeros((vol, 8), dtype=np.int32)
    sign = np.zeros((vol, 8), dtype=np.int8)
    nbr[eo] = eo[nbr_lex]
    sign[eo] = sign_lex
    return eo, nbr, sign

"""NumPy emulation of one exported tile pass, for CPU tests of the planner.

Reads the pass description exported through the C ABI (sd_plan_export_pass)
and applies it to a small state vector exactly as described in the header:
gather the tile, multiply by i^{q(y)} (-1)^{popcount(y & z_sign)}, Walsh-Hadamard over the rho span
coordinates, multiply by exp(-i tau Lambda) 2^-rho, Walsh-Hadamard, multiply by
the conjugate phase, scatter.  It is test code: it checks the planner's arithmetic
against the oracle before any GPU run; it is not the GPU path.
"""
import numpy as np


def _parity(v):
    v = np.asarray(v, dtype=np.uint64)
    out = np.zeros(v.shape, dtype=np.int64)
    w = v.copy()
    while np.any(w):
        out ^= (w & np.uint64(1)).astype(np.int64)
        w >>= np.uint64(1)
    return out


def _wht(a, rho, axis_len):
    # a: (tiles, 2^D) ; butterflies over tile-coordinate bits 0..rho-1
    a = a.copy()
    for b in range(rho):
        idx = np.arange(axis_len)
        lo = idx[(idx >> b) & 1 == 0]
        hi = lo | (1 << b)
        x, y = a[:, lo].copy(), a[:, hi].copy()
        a[:, lo] = x + y
        a[:, hi] = x - y
    return a


def apply_pass(psi, n, ps, tau):
    D, rho = ps["tile_log2"], ps["rho"]
    free = [q for q in range(n) if (ps["free_mask"] >> q) & 1]
    assert len(free) == n - D
    size = 1 << D
    tiles = 1 << (n - D)
    pv = [int(v) for v in ps["pivot_vec"]]
    pc = [int(v) for v in ps["pivot_coord"]]
    # in-tile offsets and tile coordinates of pivot pattern p
    off = np.zeros(size, dtype=np.int64)
    tc = np.zeros(size, dtype=np.int64)
    for p in range(size):
        o = t = 0
        for i in range(D):
            if (p >> i) & 1:
                o ^= pv[i]
                t ^= pc[i]
        off[p], tc[p] = o, t
    assert sorted(tc.tolist()) == list(range(size))
    xT = np.zeros(tiles, dtype=np.int64)
    for ti in range(tiles):
        xT[ti] = sum(((ti >> i) & 1) << free[i] for i in range(len(free)))
    addr = np.zeros((tiles, size), dtype=np.int64)
    addr[:, tc] = xT[:, None] ^ off[None, :]
    assert sorted(addr.ravel().tolist()) == list(range(1 << n))
    a = psi[addr].astype(np.complex128)
    t = np.arange(size)
    rmask = (1 << rho) - 1
    B = [int(v) for v in ps["cz_s"]]
    q = np.zeros(size, dtype=np.int64)
    for i in range(rho):
        yi = (t >> i) & 1
        q += yi * np.array([bin(int(B[i]) & (int(tt) & rmask)).count("1") for tt in t])
    zs = int(ps.get("z_sign", 0)) & rmask
    q += 2 * np.array([bin(int(tt) & zs).count("1") for tt in t])
    ph = (1j) ** (q % 4)
    a = a * ph[None, :]
    a = _wht(a, rho, size)
    zeta = [int(v) for v in ps["zeta"]]
    zt = [int(v) for v in ps["ztile"]]
    coef = np.asarray(ps["coef"], dtype=np.float64)
    phi = np.zeros((tiles, size))
    for k in range(len(coef)):
        sgn_tile = np.array([(-1.0) ** bin(int(x) & zt[k]).count("1") for x in xT])
        sgn_t = np.array([(-1.0) ** bin(int(tt) & zeta[k]).count("1") for tt in t])
        phi += coef[k] * sgn_tile[:, None] * sgn_t[None, :]
    a = a * np.exp(-1j * tau * phi) * 2.0 ** (-rho)
    a = _wht(a, rho, size)
    a = a * np.conj(ph)[None, :]
    out = np.array(psi, dtype=np.complex128, copy=True)
    out[addr] = a
    return out


def evolve(psi, n, passes, group_of_pass, n_groups, dt, steps, order):
    if order == 1 or n_groups == 1:
        seq = [(g, 1.0) for g in range(n_groups)]
    else:
        seq = [(g, .5) for g in range(n_groups - 1)] + [(n_groups - 1, 1.0)] + \
            [(g, .5) for g in range(n_groups - 2, -1, -1)]
    by_group = {}
    for i, g in enumerate(group_of_pass):
        by_group.setdefault(g, []).append(i)
    for _ in range(steps):
        for g, f in seq:
            for i in by_group.get(g, []):
                psi = apply_pass(psi, n, passes[i], dt * f)
    return psi

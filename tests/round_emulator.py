"""NumPy emulation of the register-round tile kernel, for CPU tests.

It follows the GPU kernel's data movement step by step, vectorised over the
threads of a block: each thread holds 16 amplitudes; in the round of chunk r
they differ in the tile coordinates reg[r]; between rounds the tile goes
through an on-chip array indexed by the swizzled slot of its tile coordinate.
The CZ/S layer is not multiplied in: its S factors are i twiddles inside the
butterflies, and its Z factors and cross-chunk CZ factors are XORs of the
addresses a forward round writes to and the mirrored inverse round reads from
(and of the coordinates that sign Lambda's terms in the Lambda round).  The
result must equal the plain description of the pass (tile_emulator), i.e. the
oracle.  Test code only; it is not the GPU path.
"""
import numpy as np


def lds_slot(t):
    t = np.asarray(t, dtype=np.int64)
    h = t >> 3
    h = h ^ (h >> 3) ^ (h >> 6) ^ (h >> 9)
    return t ^ (h & 7)


def _popc(v):
    v = np.asarray(v, dtype=np.int64)
    out = np.zeros(v.shape, dtype=np.int64)
    w = v.copy()
    while np.any(w):
        out += w & 1
        w >>= 1
    return out


def _stage(R, L, tw, fwd):
    for j in range(16):
        if (j >> L) & 1:
            continue
        k = j | (1 << L)
        a, c = R[:, j].copy(), R[:, k].copy()
        w = 1j if tw else 1.0
        if fwd:
            R[:, j] = a + w * c
            R[:, k] = a - w * c
        else:
            R[:, j] = a + c
            R[:, k] = np.conj(w) * (a - c)


def _stages(R, nb, tw, fwd):
    for L in range(nb):
        _stage(R, L, (tw >> L) & 1, fwd)


def apply_pass(psi, n, ps, rv, tau):
    """One tile pass: ps from sd_plan_export_pass, rv from sd_plan_export_rounds."""
    D, rho, c = ps["tile_log2"], ps["rho"], ps["coalesce_log2"]
    TL = D - 4
    T = 1 << TL
    tid = np.arange(T, dtype=np.int64)
    pv = [int(v) for v in ps["pivot_vec"]]
    mr = [int(v) for v in ps["pivot_coord"]]
    B = [int(v) for v in ps["cz_s"]]
    zeta = np.array([int(v) for v in ps["zeta"]], dtype=np.int64)
    ztile = [int(v) for v in ps["ztile"]]
    coef = np.asarray(ps["coef"], dtype=np.float64)
    nr = rv["n_rounds"]
    nrounds = max(nr, 1)
    free = [q for q in range(n) if (ps["free_mask"] >> q) & 1]
    # scatter/gather maps: element j of thread t is pivot pattern t + (j << TL)
    off = np.zeros((T, 16), dtype=np.int64)
    tc = np.zeros((T, 16), dtype=np.int64)
    for j in range(16):
        p = tid + (j << TL)
        for i in range(D):
            bit = (p >> i) & 1
            off ^= 0  # keep shapes
            off[:, j] ^= bit * pv[i]
            tc[:, j] ^= bit * mr[i]
    # per-thread round addresses
    rd = np.zeros((nrounds, T), dtype=np.int64)
    wr = np.zeros((nrounds, T), dtype=np.int64)
    sgnb = None
    for r in range(nrounds):
        regm = 0
        for b in range(4):
            regm |= 1 << rv["reg"][r][b]
        bt = np.zeros(T, dtype=np.int64)
        i = 0
        for q in range(D):
            if not (regm >> q) & 1:
                bt |= ((tid >> i) & 1) << q
                i += 1
        pm = np.zeros(T, dtype=np.int64)
        for l in range(4):
            if (rv["bmask"][r] >> l) & 1:
                a = rv["reg"][r][l]
                bit = (_popc(B[a] & rv["later"][r] & bt) ^ (rv["dflag"][r] >> l)) & 1
                pm |= bit << a
        rd[r] = lds_slot(bt)
        if r == nrounds - 1:
            sgnb = bt ^ pm
            wr[r] = rd[r]
        else:
            wr[r] = lds_slot(bt ^ pm)
    rs = [[int(lds_slot(1 << rv["reg"][r][b])) for b in range(4)] for r in range(4)]
    bucket = rv["bucket"]
    scale = 2.0 ** (-rho)
    out = np.array(psi, dtype=np.complex128, copy=True)
    lds = np.zeros(1 << D, dtype=np.complex128)
    for ti in range(1 << (n - D)):
        xT = 0
        for i, q in enumerate(free):
            if (ti >> i) & 1:
                xT |= 1 << q
        lds[lds_slot(tc)] = out[xT ^ off]
        cks = np.array([(-1.0 if bin(zt & xT).count("1") & 1 else 1.0) * cf
                        for zt, cf in zip(ztile, coef)])
        total = 2 * nr - 1 if nr > 0 else 1
        for step in range(total):
            r = step if step < nrounds else 2 * nr - 2 - step
            lam = step == nrounds - 1
            fwd = step < nrounds - 1
            ra = rd[r] if (fwd or lam) else wr[r]
            wa = wr[r] if fwd else rd[r]
            R = np.zeros((T, 16), dtype=np.complex128)
            for g in range(16):
                a = ra.copy()
                for b in range(4):
                    if (g >> b) & 1:
                        a ^= rs[r][b]
                R[:, g] = lds[a]
            nb = bin(rv["bmask"][r]).count("1")
            tw = rv["iflag"][r]
            if lam:
                _stages(R, nb, tw, True)
                S = np.zeros((T, 16))
                for w in range(16):
                    for k in range(bucket[w], bucket[w + 1]):
                        sg = np.where(_popc(zeta[k] & sgnb) & 1, -1.0, 1.0)
                        S[:, w] += sg * cks[k]
                A = S.copy()
                for b in range(4):
                    for j in range(16):
                        if not (j >> b) & 1:
                            a0, a1 = A[:, j].copy(), A[:, j | (1 << b)].copy()
                            A[:, j], A[:, j | (1 << b)] = a0 + a1, a0 - a1
                R = R * np.exp(-1j * tau * A) * scale
                _stages(R, nb, tw, False)
            elif fwd:
                _stages(R, nb, tw, True)
            else:
                _stages(R, nb, tw, False)
            for g in range(16):
                a = wa.copy()
                for b in range(4):
                    if (g >> b) & 1:
                        a ^= rs[r][b]
                lds[a] = R[:, g]
        out[xT ^ off] = lds[lds_slot(tc)]
    return out


def evolve(psi, n, passes, rounds, n_groups, dt, steps, order):
    if order == 1 or n_groups == 1:
        seq = [(g, 1.0) for g in range(n_groups)]
    else:
        seq = [(g, .5) for g in range(n_groups - 1)] + [(n_groups - 1, 1.0)] + \
            [(g, .5) for g in range(n_groups - 2, -1, -1)]
    by_group = {}
    for i, ps in enumerate(passes):
        by_group.setdefault(ps["group"], []).append(i)
    for _ in range(steps):
        for g, f in seq:
            for i in by_group.get(g, []):
                psi = apply_pass(psi, n, passes[i], rounds[i], dt * f)
    return psi

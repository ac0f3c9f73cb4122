"""NumPy emulation of the register-round tile kernel, for CPU tests.

It follows the GPU kernel's data movement step by step, vectorised over the
threads of a block: each thread holds 16 amplitudes; in the round of chunk r
they differ in the tile coordinates reg[r]; between rounds the tile goes
through an on-chip array indexed by the swizzled slot of its tile coordinate.
A round transforms up to 4 register coordinates, exchanges register bits 2,
3 with lane bits 4, 5 (a lane permute inside the wave) and transforms the 2
coordinates brought in.  Round 0 takes its amplitudes from the state vector
directly and its inverse round writes them back directly; when its lanes
(the lowest address bits) have components along its own coordinates, its
outputs are laid out without them and take the matching sign.
The CZ/S layer is not multiplied in: its S factors are i twiddles inside the
butterflies, and its Z factors and cross-chunk CZ factors are XORs of the
addresses a forward round writes to and the mirrored inverse round reads from
(and of the coordinates that sign Lambda's terms in the Lambda round).  The
result must equal the plain description of the pass (tile_emulator), i.e. the
oracle.  Test code only; it is not the GPU path.
"""
import numpy as np


def lds_slot(t, swz):
    t = np.asarray(t, dtype=np.int64)
    low = np.zeros(t.shape, dtype=np.int64)
    for j in range(len(swz)):
        low |= (_popc(t & swz[j]) & 1) << j
    return t ^ low


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


def _exchange(R, B, LB):
    """Register bit B <-> lane bit LB: for each register pair (j, j | 2^B) a
    2x2 transpose with the two lane halves (the lane permute of the kernel:
    new x = x on lanes with bit LB clear, y of the partner lane otherwise;
    new y = x of the partner lane where bit LB is clear, y otherwise)."""
    T = R.shape[0]
    t = np.arange(T)
    hi = ((t >> LB) & 1).astype(bool)
    partner = t ^ (1 << LB)
    for j in range(16):
        if (j >> B) & 1:
            continue
        k = j | (1 << B)
        x, y = R[:, j].copy(), R[:, k].copy()
        R[:, j] = np.where(hi, y[partner], x)
        R[:, k] = np.where(hi, y, x[partner])


def _xchg(R, nx):
    if nx >= 1:
        _exchange(R, 2, 4)
    if nx == 2:
        _exchange(R, 3, 5)


def _stages_x(R, nx):
    for L in range(2, 2 + nx):
        _stage(R, L, 0, True)


def apply_pass(psi, n, ps, rv, tau):
    """One tile pass: ps from sd_plan_export_pass, rv from sd_plan_export_rounds."""
    D, rho = ps["tile_log2"], ps["rho"]
    TL = D - 4
    T = 1 << TL
    tid = np.arange(T, dtype=np.int64)
    B = [int(v) for v in ps["cz_s"]]
    zeta = np.array([int(v) for v in ps["zeta"]], dtype=np.int64)
    ztile = [int(v) for v in ps["ztile"]]
    coef = np.asarray(ps["coef"], dtype=np.float64)
    nr = rv["n_rounds"]
    nrounds = max(nr, 1)
    free = [q for q in range(n) if (ps["free_mask"] >> q) & 1]
    basis = [int(v) for v in ps["basis"]]
    swz = rv["swz"]

    def phys(y):
        y = np.asarray(y, dtype=np.int64)
        out = np.zeros(y.shape, dtype=np.int64)
        for k in range(D):
            out ^= ((y >> k) & 1) * basis[k]
        return out

    def base(vecs):
        b = np.zeros(T, dtype=np.int64)
        for i in range(TL):
            b ^= ((tid >> i) & 1) * vecs[i]
        return b

    staged = bool(rv.get("staged", 0))
    if staged:
        # pivot order: element j of thread t is pivot pattern t + (j << TL)
        pvv = [int(v) for v in ps["pivot_vec"]]
        pcc = [int(v) for v in ps["pivot_coord"]]
        soff = np.zeros((T, 16), dtype=np.int64)
        stc = np.zeros((T, 16), dtype=np.int64)
        for j in range(16):
            pp = tid + (j << TL)
            for i in range(D):
                bit = (pp >> i) & 1
                soff[:, j] ^= bit * pvv[i]
                stc[:, j] ^= bit * pcc[i]
        sslot = lds_slot(stc, swz)
    # round 0: element g of thread t is tile coordinate bt0(t) ^ reg pattern g
    bt0 = base(rv["lanes"][0])
    y0 = np.zeros((T, 16), dtype=np.int64)
    for g in range(16):
        y0[:, g] = bt0
        for b in range(4):
            if (g >> b) & 1:
                y0[:, g] ^= 1 << rv["reg"][0][b]
    assert sorted(y0.ravel().tolist()) == list(range(1 << D))
    off = phys(y0)
    # round 0 with low-bit lanes that have components d(t) along its own
    # coordinates: its outputs are laid out without them (lanes_post[0]) and,
    # when it is not Lambda's round, carry the sign (-1)^{k.d(t)}
    # With a CZ or S among round 0's register coordinates the shift also
    # moves the outputs by m0(t) = M d(t) (M: the CZ/S form on those
    # coordinates) and adds the constant (-1)^{Q(d)}.
    sign0 = None
    m0 = np.zeros(T, dtype=np.int64)
    if rv.get("shift0", 0) and not staged:
        d = np.zeros(T, dtype=np.int64)
        for i in range(min(4, TL)):
            d ^= ((tid >> i) & 1) * (rv["lanes"][0][i] ^ rv["lanes_post"][0][i])
        nb0 = bin(rv["bmask"][0]).count("1")
        regm = sum(1 << rv["reg"][0][l] for l in range(nb0))
        qd = np.zeros(T, dtype=np.int64)
        for l in range(nb0):
            a = rv["reg"][0][l]
            m0 |= (_popc(B[a] & regm & d) & 1) << a
            higher = regm & ~((2 << a) - 1)
            qd ^= ((d >> a) & 1) & _popc(B[a] & higher & d)
        w = np.zeros(T, dtype=np.int64)
        for l in range(4):
            w |= ((d >> rv["regpost"][0][l]) & 1) << l
        kap = qd & 1
        for x in range(rv["nx"][0]):
            kap ^= (tid >> (4 + x)) & (d >> rv["reg"][0][2 + x]) & 1
        if nr >= 2:
            sign0 = np.ones((T, 16))
            for g in range(16):
                sign0[:, g] = np.where((_popc(g & w) ^ kap) & 1, -1.0, 1.0)
    # per-thread round addresses
    rd = np.zeros((nrounds, T), dtype=np.int64)
    wr = np.zeros((nrounds, T), dtype=np.int64)
    sgnb = None
    for r in range(nrounds):
        bt = base(rv["lanes"][r])
        btp = base(rv["lanes_post"][r])
        pm = np.zeros(T, dtype=np.int64)
        for l in range(6):
            if l < 4:
                if not (rv["bmask"][r] >> l) & 1:
                    continue
                a = rv["reg"][r][l]
            elif l - 4 < rv["nx"][r]:
                a = rv["xl"][r][l - 4]
            else:
                continue
            bit = (_popc(B[a] & rv["later"][r] & bt) ^ (rv["dflag"][r] >> l)) & 1
            pm |= bit << a
        if r == 0:
            btp = btp ^ m0
        rd[r] = lds_slot(bt, swz)
        if r == nrounds - 1:
            sgnb = btp ^ pm
            wr[r] = rd[r]
        else:
            wr[r] = lds_slot(btp ^ pm, swz)
    rs_pre = [[int(lds_slot(1 << rv["reg"][r][b], swz)) for b in range(4)] for r in range(4)]
    rs_post = [[int(lds_slot(1 << rv["regpost"][r][b], swz)) for b in range(4)] for r in range(4)]
    bucket = rv["bucket"]
    scale = 2.0 ** (-rho)
    out = np.array(psi, dtype=np.complex128, copy=True)
    lds = np.zeros(1 << D, dtype=np.complex128)

    def addr(start, offs):
        a = np.zeros((T, 16), dtype=np.int64)
        for g in range(16):
            a[:, g] = start
            for b in range(4):
                if (g >> b) & 1:
                    a[:, g] ^= offs[b]
        return a

    for ti in range(1 << (n - D)):
        xT = 0
        for i, q in enumerate(free):
            if (ti >> i) & 1:
                xT |= 1 << q
        cks = np.array([(-1.0 if bin(zt & xT).count("1") & 1 else 1.0) * cf
                        for zt, cf in zip(ztile, coef)])
        total = 2 * nr - 1 if nr > 0 else 1
        if staged:
            lds[sslot] = out[xT ^ soff]
        for step in range(total):
            r = step if step < nrounds else 2 * nr - 2 - step
            lam = step == nrounds - 1
            fwd = step < nrounds - 1
            last = step == total - 1
            ra = rd[r] if (fwd or lam) else wr[r]
            wa = wr[r] if fwd else rd[r]
            rin = rs_pre[r] if (fwd or lam) else rs_post[r]
            rout = rs_post[r] if fwd else rs_pre[r]
            if step == 0 and not staged:
                R = out[xT ^ off].astype(np.complex128)
            else:
                R = lds[addr(ra, rin)]
            nb = bin(rv["bmask"][r]).count("1")
            nx = rv["nx"][r]
            tw = rv["iflag"][r] & 1
            czm = rv.get("czmask", [0, 0, 0, 0])[r]
            czs = np.array([-1.0 if (czm >> g) & 1 else 1.0 for g in range(16)])
            if not lam:
                if sign0 is not None and r == 0 and last:
                    R = R * sign0
                if fwd:
                    R = R * czs
                for L in range(nb):
                    _stage(R, L, 0, True)
                _xchg(R, nx)
                _stages_x(R, nx)
                if not fwd:
                    R = R * czs
                if sign0 is not None and r == 0 and step == 0:
                    R = R * sign0
            else:
                R = R * czs
                if nb:
                    _stage(R, 0, tw, True)
                    for L in range(1, nb):
                        _stage(R, L, 0, True)
                    _xchg(R, nx)
                    _stages_x(R, nx)
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
                if nb:
                    _stages_x(R, nx)
                    _xchg(R, nx)
                    for L in range(1, nb):
                        _stage(R, L, 0, False)
                    _stage(R, 0, tw, False)
                R = R * czs
            if last and not staged:
                out[xT ^ off] = R
            else:
                lds[addr(wa, rout)] = R
        if staged:
            out[xT ^ soff] = lds[sslot]
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

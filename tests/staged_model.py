"""Test infrastructure: a numpy model of the LDS-staged schedule tables (the records that the staged
kernels read), used by the CPU tests of the scheduler.

* `load_tables` reads what tests/sched_dump.cpp writes (the host scheduler's output).
* `run_schedule` applies the tables to a state by global index: per pass and block, per stage the
  register/thread layout, per round the op lists in the kernels' order with their conditions, fused
  flips and diagonal factors, and the stage-end swap. Comparing it with the oracle checks the
  scheduler's decomposition without a GPU.
* `check_half_exchanges` simulates, slot by slot, every LDS round trip of a half-buffer pass (two
  halves split by a bit at the same thread position in both layouts; slots with the split bit
  squeezed out and one pad slot per 2^P) and checks that no two elements share a slot and every read
  returns the element the next layout expects.
* `check_wave_barriers` follows, wavefront by wavefront, the control flow of the wave-split kernel
  (its barriers sit in branches that are uniform per wavefront but differ between the two halves)
  and checks that every wavefront passes the same number of barriers and that, with the k-th
  barrier of each wavefront taken as one barrier instance, every LDS write of a round trip is
  ordered before the reads that need it and every read before the writes that overwrite it.
"""
import numpy as np

KL = 8  # op lists per register bit: 0 plain, 1 block flip, 2..5 pair flips, 6 lane flip, 7 condition
PASS = np.dtype([('m', '<i4'), ('sb', '<i4'), ('se', '<i4'), ('direct', '<i4'), ('R', 'u1', 16)])
STAGE = np.dtype([('rb0', '<i4'), ('rb1', '<i4'), ('rb', 'u1', 8), ('tb', 'u1', 16), ('sp', '<i4'), ('sq', '<i4'),
                  ('slcm', '<u4'), ('hb_in', 'u1'), ('hj_in', 'u1'), ('hb_out', 'u1'), ('hj_out', 'u1'),
                  ('sgcm', '<u8'), ('prb', 'u1', 8), ('ptb', 'u1', 16)])
MAXPAIRS = 10  # pair lists for up to 5 register bits
ROUND = np.dtype([('seg', '<i4', KL * 5 + 4), ('pseg', '<i4', MAXPAIRS + 1)])
BLK = np.dtype([('m', '<f8', 32), ('mf', '<f4', 32)])
OP = np.dtype([('pmask', '<u4'), ('lcm_t', '<u4'), ('gcm', '<u8'), ('gtb', '<u8'), ('m0', '<u4'), ('m1', '<u4'),
               ('lt', '<i4'), ('angles', '<i4'), ('m', '<f8', 8), ('theta', '<f8', 2), ('mf', '<f4', 8), ('galt', '<u8'),
               ('amask', '<u4'), ('alt_lcm', '<u4'), ('alt_col', '<u4'), ('alt_rank', '<i4')])


def npairs(le):
    return le * (le - 1) // 2


def pair_index(le, ja, jb):
    return ja * (2 * le - ja - 1) // 2 + (jb - ja - 1)


def load_tables(path):
    """(passes, stages, rounds, ops, two-qubit blocks) as written by tests/sched_dump.cpp."""
    b = open(path, 'rb').read()
    head = np.frombuffer(b[:80], '<u8')
    sizes, counts = [int(v) for v in head[:5]], [int(v) for v in head[5:]]
    assert sizes == [PASS.itemsize, STAGE.itemsize, ROUND.itemsize, OP.itemsize, BLK.itemsize], sizes
    off, out = 80, []
    for dt, c in zip((PASS, STAGE, ROUND, OP, BLK), counts):
        out.append(np.frombuffer(b, dt, c, off).copy())
        off += dt.itemsize * c
    P, S, RD, O, B = out
    for o in O:  # factors of angle-defined diagonal ops, as the device fills them in
        if o['angles'] == 1:
            o['m'][0:4] = [1.0, 0.0, np.cos(o['theta'][0]), np.sin(o['theta'][0])]
        elif o['angles'] == 3:
            th = o['theta'][0] * np.ldexp(2 * np.pi, -int(o['theta'][1]))
            o['m'][0:4] = [1.0, 0.0, np.cos(th), np.sin(th)]
        elif o['angles'] == 2:
            o['m'][0:4] = [np.cos(o['theta'][0]), np.sin(o['theta'][0]), np.cos(o['theta'][1]), np.sin(o['theta'][1])]
    return P, S, RD, O, B


def _layout(st, m, le):
    lt = m - le
    t = np.arange(1 << lt)
    et = np.zeros(1 << lt, dtype=np.int64)
    for j in range(lt):
        et |= ((t >> j) & 1) << int(st['tb'][j])
    er = np.zeros(1 << le, dtype=np.int64)
    for r in range(1 << le):
        for j in range(le):
            if (r >> j) & 1:
                er[r] |= 1 << int(st['rb'][j])
    return et, er


def _apply_dense(X, op, j, le, et, base, kind, flip_bit):
    """One dense op on register bit j. kind: 'plain', 'flip' (block/pair/lane fused flip), 'cond'."""
    mm = op['m']
    u = np.array([[mm[0] + 1j * mm[1], mm[2] + 1j * mm[3]], [mm[4] + 1j * mm[5], mm[6] + 1j * mm[7]]])
    if kind != 'cond':  # those lists hold 2x2s with a real first column; the kernels do not read u00/u10 im
        u[0, 0], u[1, 0] = mm[0], mm[4]
    if kind == 'cond' and (base & int(op['gcm'])) != int(op['gcm']):
        return
    lane_ok = (et & int(op['lcm_t'])) == int(op['lcm_t']) if kind == 'cond' else np.ones(len(et), bool)
    for r in range(1 << le):
        if (r >> j) & 1:
            continue
        p = (r & ((1 << j) - 1)) | ((r >> (j + 1)) << j)
        if kind == 'cond' and not (int(op['pmask']) >> p) & 1:
            continue
        r1 = r | (1 << j)
        a0, a1 = X[:, r].copy(), X[:, r1].copy()
        n0 = u[0, 0] * a0 + u[0, 1] * a1
        n1 = u[1, 0] * a0 + u[1, 1] * a1
        if kind == 'flip':
            if flip_bit is not None:  # per pair: the pairs with register bit flip_bit set
                neg = np.full(len(et), bool((r >> flip_bit) & 1))
            else:
                blk_ok = (base & int(op['galt'])) == int(op['galt'])
                neg = np.full(len(et), blk_ok and bool((int(op['amask']) >> p) & 1))
                neg &= (et & int(op['alt_lcm'])) == int(op['alt_lcm'])
            if op['alt_col']:
                n0 = np.where(neg, u[0, 0] * a0 - u[0, 1] * a1, n0)
                n1 = np.where(neg, u[1, 0] * a0 - u[1, 1] * a1, n1)
            else:
                n1 = np.where(neg, -n1, n1)
        X[:, r] = np.where(lane_ok, n0, a0)
        X[:, r1] = np.where(lane_ok, n1, a1)


def _apply_pair(X, blk, ja, jb, le):
    """A two-qubit block on register bits ja < jb: each group of four elements times the 4x4."""
    M = (blk['m'][0::2] + 1j * blk['m'][1::2]).reshape(4, 4)
    for r0 in range(1 << le):
        if (r0 >> ja) & 1 or (r0 >> jb) & 1:
            continue
        idx = [r0, r0 | (1 << ja), r0 | (1 << jb), r0 | (1 << ja) | (1 << jb)]
        X[:, idx] = X[:, idx] @ M.T


def run_schedule(psi, n, m, le, P, S, RD, O, B):
    psi = psi.copy()
    for ps in P:
        R = [int(v) for v in ps['R'][:m]]
        nonres = [q for q in range(n) if q not in R]
        e = np.arange(1 << m)
        loc = np.zeros(1 << m, dtype=np.int64)
        for s_, q in enumerate(R):
            loc |= ((e >> s_) & 1) << q
        for b in range(1 << (n - m)):
            base = 0
            for k, q in enumerate(nonres):
                base |= ((b >> k) & 1) << q
            idx = base | loc
            blk = psi[idx].copy()
            for si in range(ps['sb'], ps['se']):
                st = S[si]
                et, er = _layout(st, m, le)
                X = blk[et[:, None] | er[None, :]].copy()
                for ri in range(st['rb0'], st['rb1']):
                    seg = RD[ri]['seg']
                    for j in range(le):
                        for lst in range(KL):
                            for oi in range(seg[KL * j + lst], seg[KL * j + lst + 1]):
                                op = O[oi]
                                if lst == 0:
                                    _apply_dense(X, op, j, le, et, base, 'plain', None)
                                elif lst == KL - 1:
                                    _apply_dense(X, op, j, le, et, base, 'cond', None)
                                elif 2 <= lst <= 5:
                                    i = lst - 2
                                    kb = i if i < j else i + 1
                                    assert int(op['alt_rank']) == kb
                                    _apply_dense(X, op, j, le, et, base, 'flip', kb)
                                else:
                                    _apply_dense(X, op, j, le, et, base, 'flip', None)
                    for ja in range(le):  # two-qubit blocks, after the register-bit lists
                        for jb in range(ja + 1, le):
                            pseg = RD[ri]['pseg']
                            sl = pair_index(le, ja, jb)
                            for bi in range(pseg[sl], pseg[sl + 1]):
                                _apply_pair(X, B[bi], ja, jb, le)
                    for oi in range(seg[KL * le], seg[KL * le + 2]):  # sign flips, then other diagonal ops
                        op = O[oi]
                        if (base & int(op['gcm'])) != int(op['gcm']):
                            continue
                        mm = op['m']
                        d0, d1 = mm[0] + 1j * mm[1], mm[2] + 1j * mm[3]
                        lane_ok = (et & int(op['lcm_t'])) == int(op['lcm_t'])
                        f0 = np.full(len(et), d0)
                        f1 = np.full(len(et), d1)
                        if op['lt'] >= 0:
                            f1 = np.where(((et >> int(op['lt'])) & 1) == 1, d1, d0)
                        elif op['gtb']:
                            f1 = np.full(len(et), d1 if (base & int(op['gtb'])) else d0)
                        f0 = np.where(lane_ok, f0, 1)
                        f1 = np.where(lane_ok, f1, 1)
                        for r in range(1 << le):
                            if (int(op['m1']) >> r) & 1:
                                X[:, r] *= f1
                            if (int(op['m0']) >> r) & 1:
                                X[:, r] *= f0
                d = et[:, None] | er[None, :]
                if st['sp'] >= 0 and (base & int(st['sgcm'])) == int(st['sgcm']):
                    p_, q_ = int(st['sp']), int(st['sq'])
                    sel = ((d & int(st['slcm'])) == int(st['slcm'])) & ((((d >> p_) ^ (d >> q_)) & 1) == 1)
                    d = np.where(sel, d ^ ((1 << p_) | (1 << q_)), d)
                blk[d] = X
            psi[idx] = blk
    return psi


def _slot(e, P):
    return e + (e >> P)


def _squeeze(v, b):
    low = (1 << b) - 1
    return (v & low) | ((v >> 1) & ~low)


def _exchange(A, B, b, j, m, le, P):
    lt = m - le
    t = np.arange(1 << lt)
    nslots = (1 << (m - 1)) + ((1 << (m - 1)) >> P)
    mine = (t >> j) & 1
    for half in (0, 1):
        buf = np.full(nslots, -1, dtype=np.int64)
        th = t[mine == half]
        w_idx = A[0][th][:, None] | A[1][None, :]
        w_slot = _slot(_squeeze(A[0][th], b), P)[:, None] + _slot(_squeeze(A[1], b), P)[None, :]
        assert (((w_idx >> b) & 1) == half).all(), 'an element outside its half'
        assert 0 <= w_slot.min() and w_slot.max() < nslots, 'slot out of range'
        assert len(np.unique(w_slot)) == w_slot.size, 'two elements in one slot'
        buf[w_slot.ravel()] = w_idx.ravel()
        r_idx = B[0][th][:, None] | B[1][None, :]
        r_slot = _slot(_squeeze(B[0][th], b), P)[:, None] + _slot(_squeeze(B[1], b), P)[None, :]
        assert r_slot.max() < nslots, 'read slot out of range'
        assert (buf[r_slot] == r_idx).all(), 'a read returned the wrong element'


def check_half_exchanges(P, S, m, le, c128):
    """Returns (passes with a half-size buffer, those with wave-level splits)."""
    Pb = 4 if c128 else 5
    lt = m - le
    t = np.arange(1 << lt, dtype=np.int64)
    load = (t, np.arange(1 << le, dtype=np.int64) << lt)
    nhalf = nwave = 0
    for ps in P:
        if not ps['direct'] & 4:
            continue
        nhalf += 1
        sts = [S[i] for i in range(ps['sb'], ps['se'])]
        js = []
        for st in sts:
            rb = set(int(x) for x in st['rb'][:le])
            assert sorted(int(x) for x in st['tb'][:lt]) == sorted(set(range(m)) - rb)
        lays = [_layout(st, m, le) for st in sts]
        if not ps['direct'] & 1:
            _exchange(load, lays[0], int(sts[0]['hb_in']), int(sts[0]['hj_in']), m, le, Pb)
            js.append(int(sts[0]['hj_in']))
        for k in range(len(sts) - 1):
            assert sts[k]['hb_out'] == sts[k + 1]['hb_in'] and sts[k]['hj_out'] == sts[k + 1]['hj_in']
            _exchange(lays[k], lays[k + 1], int(sts[k]['hb_out']), int(sts[k]['hj_out']), m, le, Pb)
            js.append(int(sts[k]['hj_out']))
        if not ps['direct'] & 2:
            _exchange(lays[-1], load, int(sts[-1]['hb_out']), int(sts[-1]['hj_out']), m, le, Pb)
            js.append(int(sts[-1]['hj_out']))
        if ps['direct'] & 8:
            assert all(j >= 6 for j in js), 'a wave-split pass with a lane-level split'
            nwave += 1
    return nhalf, nwave


def _wave_trace(ps, sts, w):
    """Events of wavefront w of a wave-split pass, in program order: ('B',) for a barrier, ('W', k) /
    ('R', k) for its LDS writes / reads of round trip k. Mirrors wave_out / wave_in: a wavefront is in
    the second half of a round trip when its bit j (a thread position >= 6) is set."""
    ev = []
    k = [0]

    def second(j):
        return (w >> (j - 6)) & 1

    def wave_out(j, pre):
        if pre:
            ev.append(('B',))
        if second(j):
            ev.extend([('B',), ('B',)])
        ev.append(('W', k[0]))
        ev.append(('B',))

    def wave_in(j):
        ev.append(('R', k[0]))
        if not second(j):
            ev.extend([('B',), ('B',)])
        k[0] += 1

    for i, st in enumerate(sts):
        first, last = i == 0, i == len(sts) - 1
        if not (first and ps['direct'] & 1):
            if first:
                wave_out(int(st['hj_in']), False)
            wave_in(int(st['hj_in']))
        if last:
            break
        wave_out(int(st['hj_out']), True)
    if not ps['direct'] & 2:
        wave_out(int(sts[-1]['hj_out']), True)
        wave_in(int(sts[-1]['hj_out']))
    return ev


def check_wave_barriers(P, S, m, le):
    """Returns the number of wave-split passes checked."""
    lt = m - le
    nw = 1 << (lt - 6)
    checked = 0
    for ps in P:
        if (ps['direct'] & 12) != 12:
            continue
        sts = [S[i] for i in range(ps['sb'], ps['se'])]
        traces = [_wave_trace(ps, sts, w) for w in range(nw)]
        nb = [sum(1 for e in t if e[0] == 'B') for t in traces]
        assert len(set(nb)) == 1, f'wavefronts pass different numbers of barriers: {nb}'
        # (wave, barriers passed before the event) of every write and read of each round trip
        W, R = {}, {}
        for w, t in enumerate(traces):
            nbar = 0
            for e in t:
                if e[0] == 'B':
                    nbar += 1
                else:
                    (W if e[0] == 'W' else R).setdefault(e[1], []).append((w, nbar))

        def before(a, b):  # a happens before b: same wavefront in program order, or a barrier between
            return (a[0] == b[0] and a[1] <= b[1]) or a[1] < b[1]

        nrt = len(W)
        assert sorted(W) == sorted(R) == list(range(nrt))
        js = []
        if not ps['direct'] & 1:
            js.append(int(sts[0]['hj_in']))
        js += [int(st['hj_out']) for st in sts[:-1]]
        if not ps['direct'] & 2:
            js.append(int(sts[-1]['hj_out']))
        assert len(js) == nrt
        for k in range(nrt):
            half = {w: (w >> (js[k] - 6)) & 1 for w in range(nw)}
            for h in (0, 1):
                ws = [e for e in W[k] if half[e[0]] == h]
                rs = [e for e in R[k] if half[e[0]] == h]
                assert all(before(a, b) for a in ws for b in rs), f'round trip {k}: a read before a write of its half'
            r0 = [e for e in R[k] if half[e[0]] == 0]
            w1 = [e for e in W[k] if half[e[0]] == 1]
            assert all(before(a, b) for a in r0 for b in w1), f'round trip {k}: the second half writes before the first reads'
            if k + 1 < nrt:
                assert all(before(a, b) for a in R[k] for b in W[k + 1]), f'round trip {k + 1} writes before {k} is read'
        checked += 1
    return checked

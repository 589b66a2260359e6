"""Matrix-product-operator (MPO) form of the electronic Hamiltonian.

Host-side problem setup (not on the timed path).  The paper takes the operator
``A`` in tensor-train form (eq. MPO) and defers its construction for the
second-quantised Hamiltonian (Section 3.2) to the literature; this module
builds one directly as a finite-state machine over operator strings.

Hamiltonian (chemists' integrals ``(pq|rs)``):

    H = sum_pq h_pq sum_s a+_{ps} a_{qs}
      + 1/2 sum_pqrs (pq|rs) sum_{s,t} a+_{ps} a+_{rt} a_{st} a_{qs}

Sites are spatial orbitals with local basis ``|0>, |up>, |dn>, |updn>``
(index ``n_up + 2 n_dn``); the Jordan-Wigner order puts alpha before beta
within a site.  Every term is rewritten as a product ordered by spin orbital
(sign from the permutation); its factor on site ``t`` is the ordered product
of its local operators there times the parity ``P = (-1)^n`` raised to the
number of its operators right of ``t``.

Channels at bond k (sites < k on the left):

* ``I``       nothing placed yet; ``H`` every operator placed;
* ``S(x)``    one operator x placed on the left (normal);
* ``P(x,y)``  two operators placed, bonds k <= m (normal pairs);
* ``Q(y,z)``  two operators y,z still to come, bonds k > m (complementary:
              the left part is the coefficient-weighted sum of left pairs);
* ``C(y)``    one operator y still to come (complementary triples and the
              one-body remainder).

Normal channels carry products of left operators with no coefficient;
a term's coefficient is applied on the transition where its channel turns
complementary.  With the switch bond ``m = L//2`` the bond dimension is about
``2 + 4L + 8 l^2`` with ``l = min(k, L-k)``.

Output per site ``k``: sparse entries ``(A, B, op[4][4])`` of
``W_k[A, s_out, s_in, B]``, and per bond the channel charges
``(dN, d2Sz)`` of the left operators.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

# local operator types: 0 = a+ alpha, 1 = a+ beta, 2 = a alpha, 3 = a beta
_CDAG_A = np.zeros((4, 4)); _CDAG_A[1, 0] = 1.0; _CDAG_A[3, 2] = 1.0
_CDAG_B = np.zeros((4, 4)); _CDAG_B[2, 0] = 1.0; _CDAG_B[3, 1] = -1.0
LOCAL_OPS = np.stack([_CDAG_A, _CDAG_B, _CDAG_A.T, _CDAG_B.T])
PARITY = np.diag([1.0, -1.0, -1.0, 1.0])
OP_CHARGE = np.array([(1, 1), (1, -1), (-1, -1), (-1, 1)], dtype=np.int64)

T_I, T_S, T_P, T_C, T_Q, T_H = 0, 1, 2, 3, 4, 5
_NORMAL = (T_I, T_S, T_P)


@dataclass
class MPO:
    L: int
    switch: int
    R: list            # bond dimensions, length L+1
    A: list            # per site: int32 [nnz]
    B: list            # per site: int32 [nnz]
    ops: list          # per site: float64 [nnz, 4, 4]
    chan_q: list       # per bond: int32 [R_k, 2]
    chan_codes: list   # per bond: int64 [R_k]

    def nnz(self):
        return [len(a) for a in self.A]

    def dense_core(self, k):
        W = np.zeros((self.R[k], 4, 4, self.R[k + 1]))
        np.add.at(W, (self.A[k], slice(None), slice(None), self.B[k]), self.ops[k])
        return W


def _terms(h, B, tol=0.0):
    """All operator strings with their coefficients.  Returns list of
    (codes[T, nops], coef[T]) with codes = 4*site + type, in the written order."""
    L = h.shape[0]
    out = []
    # one-body
    p, q, s = np.meshgrid(np.arange(L), np.arange(L), np.arange(2), indexing="ij")
    p, q, s = p.ravel(), q.ravel(), s.ravel()
    coef = h[p, q]
    keep = np.abs(coef) > tol
    codes = np.stack([4 * p + s, 4 * q + 2 + s], axis=1)[keep]
    out.append((codes, coef[keep], (p * L + q)[keep]))
    # two-body: a+_{p s} a+_{r t} a_{u t} a_{q s}, coefficient (pq|ru)/2
    eri = np.einsum("kpq,krs->pqrs", B, B)
    idx = np.nonzero(np.abs(eri) > tol)
    pp, qq, rr, uu = idx
    vals = 0.5 * eri[idx]
    for sa in range(2):
        for sb in range(2):
            ok = ~(((pp == rr) & (sa == sb)) | ((uu == qq) & (sa == sb)))
            c = np.stack([4 * pp + sa, 4 * rr + sb, 4 * uu + 2 + sb, 4 * qq + 2 + sa], axis=1)[ok]
            out.append((c, vals[ok], np.full(int(ok.sum()), -1)))
    return out


def _canonical(codes, coef):
    """Stable sort of each string by spin orbital with the fermionic sign."""
    site = codes // 4
    spin = (codes % 4) % 2
    key = 2 * site + spin
    order = np.argsort(key, axis=1, kind="stable")
    n = codes.shape[1]
    inv = np.zeros(len(codes), dtype=np.int64)
    for i in range(n):
        for j in range(i + 1, n):
            inv += key[:, i] > key[:, j]
    sign = np.where(inv % 2 == 0, 1.0, -1.0)
    return np.take_along_axis(codes, order, axis=1), coef * sign, sign


class _Coder:
    def __init__(self, L):
        self.nop = 4 * L
        self.big = self.nop * self.nop + 1

    def code(self, typ, payload):
        return typ * self.big + payload

    def typ(self, code):
        return code // self.big


def _channel(cd, typ_sel, sorted_codes, nops, nl, bond_after_switch):
    """Channel code for each term given its left count ``nl`` (vector)."""
    T = len(nl)
    out = np.empty(T, dtype=np.int64)
    o = sorted_codes
    z = nl == 0
    out[z] = cd.code(T_I, 0)
    full = nl == nops
    out[full] = cd.code(T_H, 0)
    one = (nl == 1) & ~full
    out[one] = cd.code(T_S, o[one, 0])
    if nops == 4:
        three = nl == 3
        out[three] = cd.code(T_C, o[three, 3])
        two = nl == 2
        if bond_after_switch is None:
            raise ValueError
        tq = two & bond_after_switch
        tp = two & ~bond_after_switch
        out[tp] = cd.code(T_P, o[tp, 0] * cd.nop + o[tp, 1])
        out[tq] = cd.code(T_Q, o[tq, 2] * cd.nop + o[tq, 3])
    return out


def _local_code(types, parity):
    c = np.zeros(types.shape[0], dtype=np.int64)
    for i in range(types.shape[1]):
        c += (types[:, i] + 1) * (5**i)
    return c + 625 * parity


def _local_matrix_uncached(code):
    par = code // 625
    c = code % 625
    M = np.eye(4)
    while c:
        t = c % 5 - 1
        c //= 5
        M = M @ LOCAL_OPS[t]
    if par:
        M = M @ PARITY
    return M


_LOCAL_TABLE = np.stack([_local_matrix_uncached(c).reshape(16) for c in range(1250)])


def _local_matrix(code):
    return _LOCAL_TABLE[code].reshape(4, 4)


def build_mpo(h, B, switch=None, tol=0.0) -> MPO:
    """Exact MPO of the Hamiltonian defined by ``h`` and the factors ``B``."""
    L = h.shape[0]
    m = L // 2 if switch is None else switch
    cd = _Coder(L)
    ev_site, ev_b, ev_a, ev_loc, ev_coef, ev_sw = [], [], [], [], [], []
    seg_code, seg_lo, seg_hi = [], [], []

    dh_site, dh_b, dh_a, dh_loc, dh_sign, dh_tag = [], [], [], [], [], []
    for codes, coef, tag in _terms(h, B, tol):
        if len(codes) == 0:
            continue
        nops = codes.shape[1]
        o, cf, sgn = _canonical(codes, coef)
        site = o // 4
        typ = o % 4
        T = len(o)
        ar = np.arange(T)
        prev_site = np.full(T, -1)
        # event list for this class: op-site events and the switch event
        cur_lo = np.zeros(T, dtype=np.int64)
        ev_list = []
        for i in range(nops):
            first = (site[:, i] != site[:, i - 1]) if i > 0 else np.ones(T, dtype=bool)
            cnt = np.zeros(T, dtype=np.int64)
            for j in range(i, nops):
                cnt += site[:, j] == site[:, i]
            ev_list.append((i, first, cnt))
        # switch event at site m: two ops left of m, two right of m
        if nops == 4:
            nl_m = np.sum(site < m, axis=1)
            at_m = np.any(site == m, axis=1)
            sw_ev = (nl_m == 2) & ~at_m
        else:
            sw_ev = np.zeros(T, dtype=bool)

        # collect event sites in order for segment bookkeeping
        events = []  # (sel, t, nl_before, nl_after, loc_code)
        for i, first, cnt in ev_list:
            sel = np.nonzero(first)[0]
            t = site[sel, i]
            c = cnt[sel]
            types = np.full((len(sel), 4), -1, dtype=np.int64)
            for j in range(4):
                valid = j < c
                if np.any(valid):
                    col = np.minimum(i + j, nops - 1)
                    types[valid, j] = typ[sel[valid], col[valid] if np.ndim(col) else col]
            par = (nops - (i + c)) % 2
            loc = np.zeros(len(sel), dtype=np.int64)
            for j in range(4):
                valid = types[:, j] >= 0
                loc[valid] += (types[valid, j] + 1) * (5**j)
            loc += 625 * par
            events.append((sel, t, np.full(len(sel), i), i + c, loc))
        sel = np.nonzero(sw_ev)[0]
        events.append((sel, np.full(len(sel), m), np.full(len(sel), 2), np.full(len(sel), 2),
                       np.zeros(len(sel), dtype=np.int64)))

        for sel, t, nlb, nla, loc in events:
            if len(sel) == 0:
                continue
            osub = o[sel]
            chb = _channel(cd, None, osub, nops, nlb, t > m)       # bond t
            cha = _channel(cd, None, osub, nops, nla, (t + 1) > m)  # bond t+1
            sw = np.isin(chb // cd.big, _NORMAL) & ~np.isin(cha // cd.big, _NORMAL)
            ev_site.append(t); ev_b.append(chb); ev_a.append(cha); ev_loc.append(loc)
            ev_coef.append(np.where(sw, cf[sel], 0.0)); ev_sw.append(sw)
            if nops == 2 and np.any(sw):
                dh_site.append(t[sw]); dh_b.append(chb[sw]); dh_a.append(cha[sw]); dh_loc.append(loc[sw])
                dh_sign.append(sgn[sel][sw]); dh_tag.append(tag[sel][sw])
            # the channel after the event lives on bonds t+1 .. (next event site)
            seg_code.append(cha); seg_lo.append(t + 1)
        # segment upper ends: next event site per term, computed by sorting events
        all_t = np.concatenate([np.asarray(e[1]) for e in events if len(e[0])])
        all_sel = np.concatenate([e[0] for e in events if len(e[0])])
        order = np.lexsort((all_t, all_sel))
        st, ss = all_t[order], all_sel[order]
        nxt = np.empty_like(st)
        nxt[:-1] = st[1:]
        last = np.ones(len(st), dtype=bool)
        last[:-1] = ss[1:] != ss[:-1]
        nxt[last] = L
        # map back: hi for each (event in concatenated original order)
        hi = np.empty_like(nxt)
        hi[order] = nxt
        seg_hi.append(hi)

    ev_site = np.concatenate(ev_site); ev_b = np.concatenate(ev_b); ev_a = np.concatenate(ev_a)
    ev_loc = np.concatenate(ev_loc); ev_coef = np.concatenate(ev_coef); ev_sw = np.concatenate(ev_sw)
    seg_code = np.concatenate(seg_code); seg_lo = np.concatenate(seg_lo); seg_hi = np.concatenate(seg_hi)

    # channel existence: I on bonds 0..L-1, H on 1..L, others from segments
    codes_u, inv = np.unique(seg_code, return_inverse=True)
    lo = np.full(len(codes_u), L + 1); hi = np.full(len(codes_u), -1)
    np.minimum.at(lo, inv, seg_lo)
    np.maximum.at(hi, inv, seg_hi)
    cI, cH = cd.code(T_I, 0), cd.code(T_H, 0)
    keep = (codes_u != cH)
    codes_u, lo, hi = codes_u[keep], lo[keep], hi[keep]
    codes_u = np.concatenate([[cI], codes_u, [cH]])
    lo = np.concatenate([[0], lo, [1]])
    hi = np.concatenate([[L - 1], hi, [L]])

    chan_codes, chan_q, R = [], [], []
    for k in range(L + 1):
        sel = (lo <= k) & (hi >= k)
        cc = codes_u[sel]
        chan_codes.append(cc)
        R.append(len(cc))
        chan_q.append(_channel_charge(cd, cc))

    table = _LOCAL_TABLE
    order = np.argsort(ev_site, kind="stable")
    ev_site, ev_b, ev_a, ev_loc, ev_coef, ev_sw = (ev_site[order], ev_b[order], ev_a[order], ev_loc[order],
                                                    ev_coef[order], ev_sw[order])
    bounds = np.searchsorted(ev_site, np.arange(L + 1))
    As, Bs, Ops, Keys = [], [], [], []
    loc_I, loc_P = 0, 625
    for k in range(L):
        cb, ca = chan_codes[k], chan_codes[k + 1]
        Ra = len(ca)
        # pass-through entries
        both = np.intersect1d(cb, ca)
        tb = both // cd.big
        pb = np.searchsorted(cb, both)
        pa = np.searchsorted(ca, both)
        ploc = np.where((tb == T_S) | (tb == T_C), loc_P, loc_I)
        sl = slice(bounds[k], bounds[k + 1])
        b_, a_, l_, c_, s_ = ev_b[sl], ev_a[sl], ev_loc[sl], ev_coef[sl], ev_sw[sl]
        ib = np.searchsorted(cb, b_)
        ia = np.searchsorted(ca, a_)
        # non-switch events: one fixed local operator per (b, a)
        ns = ~s_
        key_ns = np.unique((ib[ns].astype(np.int64) * Ra + ia[ns]) * 1250 + l_[ns])
        kb_ns = key_ns // 1250
        if len(np.unique(kb_ns)) != len(kb_ns):
            raise RuntimeError("conflicting MPO transition")
        all_key = np.concatenate([pb.astype(np.int64) * Ra + pa, kb_ns, ib[s_].astype(np.int64) * Ra + ia[s_]])
        all_loc = np.concatenate([ploc, key_ns % 1250, l_[s_]])
        all_cf = np.concatenate([np.ones(len(pb)), np.ones(len(kb_ns)), c_[s_]])
        keep = all_cf != 0.0
        all_key, all_loc, all_cf = all_key[keep], all_loc[keep], all_cf[keep]
        uk, inv = np.unique(all_key, return_inverse=True)
        ops = np.zeros((len(uk), 16))
        np.add.at(ops, inv.ravel(), all_cf[:, None] * table[all_loc])
        Keys.append(uk)
        As.append((uk // Ra).astype(np.int32))
        Bs.append((uk % Ra).astype(np.int32))
        Ops.append(ops.reshape(-1, 4, 4))
    mpo = MPO(L, m, R, As, Bs, Ops, chan_q, chan_codes)
    # derivative of every entry with respect to h_pq (one-body switch transitions)
    dh = []
    if dh_site:
        ds = np.concatenate(dh_site); db = np.concatenate(dh_b); da = np.concatenate(dh_a)
        dl = np.concatenate(dh_loc); dg = np.concatenate(dh_sign); dt = np.concatenate(dh_tag)
        for t_, b_, a_, l_, g_, tg in zip(ds, db, da, dl, dg, dt):
            t_ = int(t_)
            ib = np.searchsorted(chan_codes[t_], b_)
            ia = np.searchsorted(chan_codes[t_ + 1], a_)
            key = int(ib) * len(chan_codes[t_ + 1]) + int(ia)
            e = int(np.searchsorted(Keys[t_], key))
            dh.append((t_, e, int(tg) // L, int(tg) % L, g_ * _local_matrix(int(l_))))
    mpo.dh = dh
    mpo.blocks = _switch_blocks(mpo, cd)
    return mpo


def _switch_blocks(mpo, cd):
    """Per site ``(p0, p1, q0, q1)``: the coefficient block P(bond m) -> Q(bond m+1)
    at the switch site (identity local operator times the integral), else -1s."""
    out = []
    for k in range(mpo.L):
        tb = mpo.chan_codes[k] // cd.big
        ta = mpo.chan_codes[k + 1] // cd.big
        pidx = np.nonzero(tb == T_P)[0]
        qidx = np.nonzero(ta == T_Q)[0]
        if len(pidx) and len(qidx):
            p0, p1, q0, q1 = int(pidx[0]), int(pidx[-1]) + 1, int(qidx[0]), int(qidx[-1]) + 1
            assert p1 - p0 == len(pidx) and q1 - q0 == len(qidx)
            inblk = (mpo.A[k] >= p0) & (mpo.A[k] < p1) & (mpo.B[k] >= q0) & (mpo.B[k] < q1)
            ops = mpo.ops[k][inblk]
            eye = ops[:, 0, 0][:, None, None] * np.eye(4)[None]
            assert np.abs(ops - eye).max(initial=0.0) <= 1e-14 * max(1.0, np.abs(ops).max(initial=0.0))
            out.append((p0, p1, q0, q1))
        else:
            out.append((-1, -1, -1, -1))
    return out


def h_gradient(mpo, gops):
    """dE/dh_pq from per-entry gradients ``gops[k][e][4][4]`` of every MPO entry."""
    g = np.zeros((mpo.L, mpo.L))
    for k, e, p, q, D in mpo.dh:
        g[p, q] += float(np.sum(np.asarray(gops[k][e]).reshape(4, 4) * D))
    return g


def _channel_charge(cd, codes):
    q = np.zeros((len(codes), 2), dtype=np.int64)
    t = codes // cd.big
    pay = codes % cd.big
    for typ_, sgn in ((T_S, 1), (T_C, -1)):
        s = t == typ_
        q[s] = sgn * OP_CHARGE[pay[s] % 4]
    for typ_, sgn in ((T_P, 1), (T_Q, -1)):
        s = t == typ_
        o1, o2 = pay[s] // cd.nop, pay[s] % cd.nop
        q[s] = sgn * (OP_CHARGE[o1 % 4] + OP_CHARGE[o2 % 4])
    return q.astype(np.int32)


def mpo_to_matrix(mpo: MPO) -> np.ndarray:
    """Contract the MPO to the full 4^L x 4^L matrix (tiny L only)."""
    M = None
    for k in range(mpo.L):
        W = mpo.dense_core(k)  # [A, s', s, B]
        if M is None:
            M = W[0]  # [s', s, B]
            M = M.reshape(4, 4, -1)
        else:
            D = M.shape[0]
            M = np.einsum("xyA,AusB->xuysB", M, W).reshape(D * 4, D * 4, -1)
    return M[:, :, 0]

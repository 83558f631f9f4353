"""A CPU model of the fused Monolithic* level kernel's tile algorithm, for tests.

It follows the HIP kernel step by step, with the GPU's parallel structure made
explicit, so that the kernel's logic can be checked without a GPU:

* a tile of 64 x (NW * RB) quadruples; wavefront w holds tile rows
  j * NW + w (j < RB), one quadruple column per lane (a 64-vector here);
* horizontal neighbours by a lane shift that feeds 0 at the wavefront's ends
  (the DPP wave shifts);
* vertical neighbours through LDS planes [buffer][component][row][lane] that
  start as NaN, published before each spatial step, with barriers exactly
  where the kernel has them (double buffering: one per spatial step; single
  buffering: one more between a step's reads and the next publication);
* a race checker: between two barriers (an epoch) the wavefronts run in any
  order, so a plane row read by one wavefront and written by another in the
  same epoch, or written by two, is a race and raises `Race`;
* whole-sample symmetric extension by mirrored loads, the tile's centring
  constant taken from the middle row of its centring cell, output of the
  interior quadruples only.

The arithmetic runs in the dtype given (float64 to compare with the oracle,
float32 for bitwise comparisons between tile heights).  This is a model of
the kernel for the tests, written from the lifting steps (Sec. 3-4): it is
not the oracle, which is a separable lifting written from Sec. 2.
"""
import numpy as np

TX, NW = 64, 4
LL, HL, LH, HH = 0, 1, 2, 3
HALO = {"cdf53": 1, "cdf97": 2, "dd137": 3}   # quadruples of halo per side
PAD = {"cdf53": 1, "cdf97": 1, "dd137": 2}    # plane padding rows (vertical reach)
CELL = {"cdf53": 30, "cdf97": 24, "dd137": 18}
ALPHA, BETA = -1.58613434205992355842832, -0.0529801185729614146241296
GAMMA, DELTA = 0.88291107553093329591979, 0.443506852043971152115604
PAIRS = {"cdf53": [(-0.5, 0.25)], "cdf97": [(ALPHA, BETA), (GAMMA, DELTA)],
         "dd137": [(-0.5625, 0.28125)]}


class Race(AssertionError):
    pass


def predict_taps(wav, k):
    """Neighbour part P1 of pair k's predict, as (row/lane offset, coefficient)."""
    if wav == "dd137":
        return [(1, -0.5625), (-1, 0.0625), (2, 0.0625)]
    return [(1, PAIRS[wav][k][0])]


def update_taps(wav, k):
    if wav == "dd137":
        return [(-1, 0.28125), (1, -0.03125), (-2, -0.03125)]
    return [(-1, PAIRS[wav][k][1])]


def mirror(j, n):
    if 0 <= j < n:
        return j
    p = 2 * (n - 1)
    j %= p
    return p - j if j >= n else j


def lane_shift(v, d):
    """Lane i gets lane i + d; lanes past either end get 0."""
    r = np.zeros_like(v)
    if d > 0:
        r[:-d] = v[d:]
    else:
        r[-d:] = v[:d]
    return r


class Tile:
    def __init__(self, wav, rb, nb, dtype, barriers=None):
        self.wav, self.rb, self.nb, self.dt = wav, rb, nb, dtype
        self.ty = NW * rb
        self.pad = PAD[wav]
        self.q = np.zeros((NW, rb, 4, TX), dtype)
        self.planes = np.full((2, 2, self.ty + 2 * self.pad, TX), np.nan, dtype)
        # race bookkeeping per plane row: (epoch, writer), (epoch, readers)
        self.epoch = 0
        self.written = {}
        self.read = {}
        # which barriers to place (all True is the kernel's schedule)
        self.barriers = barriers or {}

    # -- LDS with the race checker ------------------------------------------
    def _key(self, b, comp, r):
        return (0 if self.nb == 1 else b, comp, r)

    def write_row(self, w, b, comp, r, v):
        key = self._key(b, comp, r)
        e, readers = self.read.get(key, (-1, set()))
        if e == self.epoch and readers - {w}:
            raise Race(f"wave {w} overwrites plane row {key} read by {readers - {w}} in epoch {e}")
        e, writer = self.written.get(key, (-1, None))
        if e == self.epoch and writer != w:
            raise Race(f"waves {writer} and {w} both write plane row {key} in epoch {e}")
        self.written[key] = (self.epoch, w)
        self.planes[key[0], comp, r + self.pad] = v

    def read_row(self, w, b, comp, r):
        key = self._key(b, comp, r)
        e, writer = self.written.get(key, (-1, None))
        if e == self.epoch and writer != w:
            raise Race(f"wave {w} reads plane row {key} written by wave {writer} in epoch {e}")
        e, readers = self.read.get(key, (-1, set()))
        self.read[key] = (self.epoch, (readers if e == self.epoch else set()) | {w})
        return self.planes[key[0], comp, r + self.pad]

    def barrier(self, name):
        if self.barriers.get(name, True):
            self.epoch += 1

    # -- the kernel's steps ---------------------------------------------------
    def row(self, j, w):
        return j * NW + w

    def publish(self, b, comps):
        for w in range(NW):
            for j in range(self.rb):
                for i, comp in enumerate(comps):
                    self.write_row(w, b, i, self.row(j, w), self.q[w, j, comp].copy())

    def taps(self, taps, f):
        acc = np.zeros(TX, self.dt)
        for o, c in taps:
            acc = acc + self.dt(c) * f(o)
        return acc

    def predict_step(self, k, inv):
        t = predict_taps(self.wav, k)
        for w in range(NW):
            for j in range(self.rb):
                r, q = self.row(j, w), self.q[w, j]
                vll = self.taps(t, lambda o: self.read_row(w, 0, 0, r + o))
                vhl = self.taps(t, lambda o: self.read_row(w, 0, 1, r + o))
                hll = self.taps(t, lambda o: lane_shift(q[LL], o))
                hlh = self.taps(t, lambda o: lane_shift(q[LH], o))
                dll = self.taps(t, lambda o: lane_shift(vll, o))
                s = -1 if inv else 1
                q[HL] += s * hll
                q[LH] += s * vll
                q[HH] += dll + s * (vhl + hlh)

    def update_step(self, k, inv):
        t = update_taps(self.wav, k)
        for w in range(NW):
            for j in range(self.rb):
                r, q = self.row(j, w), self.q[w, j]
                vlh = self.taps(t, lambda o: self.read_row(w, 1, 0, r + o))
                vhh = self.taps(t, lambda o: self.read_row(w, 1, 1, r + o))
                hhl = self.taps(t, lambda o: lane_shift(q[HL], o))
                hhh = self.taps(t, lambda o: lane_shift(q[HH], o))
                dhh = self.taps(t, lambda o: lane_shift(vhh, o))
                s = -1 if inv else 1
                q[LL] += dhh + s * (hhl + vlh)
                q[HL] += s * vhh
                q[LH] += s * hhh

    def scalar(self, kind, c):
        q, c = self.q, self.dt(c)
        if kind == "predict":      # T^H_{P0}, then T^V_{P0}
            q[:, :, HL] += c * q[:, :, LL]; q[:, :, HH] += c * q[:, :, LH]
            q[:, :, LH] += c * q[:, :, LL]; q[:, :, HH] += c * q[:, :, HL]
        elif kind == "update":     # S^H_{U0}, then S^V_{U0}
            q[:, :, LL] += c * q[:, :, HL]; q[:, :, LH] += c * q[:, :, HH]
            q[:, :, LL] += c * q[:, :, LH]; q[:, :, HL] += c * q[:, :, HH]
        elif kind == "unupdate":
            q[:, :, LL] -= c * q[:, :, LH]; q[:, :, HL] -= c * q[:, :, HH]
            q[:, :, LL] -= c * q[:, :, HL]; q[:, :, LH] -= c * q[:, :, HH]
        else:                      # unpredict
            q[:, :, HH] -= c * q[:, :, HL]; q[:, :, LH] -= c * q[:, :, LL]
            q[:, :, HH] -= c * q[:, :, LH]; q[:, :, HL] -= c * q[:, :, LL]

    def forward(self):
        for k, (p, u) in enumerate(PAIRS[self.wav]):
            if self.nb == 1 and k > 0:
                self.barrier("before_predict_publish")
            self.publish(0, (LL, HL))
            self.barrier("predict")
            self.predict_step(k, False)
            self.scalar("predict", p)
            if self.nb == 1:
                self.barrier("before_update_publish")
            self.publish(1, (LH, HH))
            self.barrier("update")
            self.update_step(k, False)
            self.scalar("update", u)

    def inverse(self):
        pairs = PAIRS[self.wav]
        for kk in range(len(pairs)):
            k = len(pairs) - 1 - kk
            p, u = pairs[k]
            self.scalar("unupdate", u)
            if self.nb == 1 and kk > 0:
                self.barrier("before_update_publish")
            self.publish(1, (LH, HH))
            self.barrier("update")
            self.update_step(k, True)
            self.scalar("unpredict", p)
            if self.nb == 1:
                self.barrier("before_predict_publish")
            self.publish(0, (LL, HL))
            self.barrier("predict")
            self.predict_step(k, True)


def unit_dc_scales(wav):
    k = 1.0
    if wav == "cdf97":
        k = 1.0 + 2.0 * BETA * (1.0 + 2.0 * ALPHA)
    return 1.0 / (k * k), k * k


def _tiles(wav, rb, w, h):
    hq = HALO[wav]
    ix, iy = TX - 2 * hq, NW * rb - 2 * hq
    qw, qh = (w + 1) // 2, (h + 1) // 2
    return hq, ix, iy, -(-qw // ix), -(-qh // iy)


def forward(img, wav, rb, nb=2, dtype=np.float64, barriers=None, shared_planes=False):
    """One forward level (UNIT_DC) of the modelled kernel: Mallat layout.
    shared_planes: one work-group runs the tiles one after another on the
    same planes, with no barrier between tiles (the fused multi-level tail);
    the race checker then spans the tiles."""
    h, w = img.shape
    img = img.astype(dtype)
    sll, shh = (dtype(v) for v in unit_dc_scales(wav))
    hq, ix, iy, ntx, nty = _tiles(wav, rb, w, h)
    qw, qh = (w + 1) // 2, (h + 1) // 2
    out = np.full((h, w), np.nan)
    shared = Tile(wav, rb, nb, dtype, barriers) if shared_planes else None
    for tr in range(nty):
        for tc in range(ntx):
            t = shared if shared is not None else Tile(wav, rb, nb, dtype, barriers)
            qc = tc * ix - hq + np.arange(TX)
            x0 = np.array([mirror(2 * c, w) for c in qc])
            x1 = np.array([mirror(2 * c + 1, w) for c in qc])

            def quad_row(qr):
                r0, r1 = mirror(2 * qr, h), mirror(2 * qr + 1, h)
                return img[r0, x0], img[r0, x1], img[r1, x0], img[r1, x1]
            cell = CELL[wav]
            c = np.rint(sum(v.sum() for v in quad_row(tr * iy // cell * cell + cell // 2)) / (4 * TX))
            c = dtype(c)
            for wv in range(NW):
                for j in range(rb):
                    for e, v in enumerate(quad_row(tr * iy - hq + j * NW + wv)):
                        t.q[wv, j, e] = v - c
            t.forward()
            for wv in range(NW):
                for j in range(rb):
                    r = j * NW + wv
                    qr = tr * iy - hq + r
                    if r < hq or r >= NW * rb - hq or qr >= qh:
                        continue
                    for lane in range(hq, TX - hq):
                        cc = qc[lane]
                        if cc >= qw:
                            continue
                        out[qr, cc] = t.q[wv, j, LL, lane] * sll + c
                        if cc < w // 2:
                            out[qr, qw + cc] = t.q[wv, j, HL, lane]
                        if qr < h // 2:
                            out[qh + qr, cc] = t.q[wv, j, LH, lane]
                            if cc < w // 2:
                                out[qh + qr, qw + cc] = t.q[wv, j, HH, lane] * shh
    return out


def inverse(coef, wav, rb, nb=2, dtype=np.float64, barriers=None, shared_planes=False):
    """One inverse level (UNIT_DC) of the modelled kernel: the image
    (shared_planes as for forward)."""
    h, w = coef.shape
    coef = coef.astype(dtype)
    sll, shh = (dtype(v) for v in unit_dc_scales(wav))
    hq, ix, iy, ntx, nty = _tiles(wav, rb, w, h)
    qw, qh = (w + 1) // 2, (h + 1) // 2
    out = np.full((h, w), np.nan)
    shared = Tile(wav, rb, nb, dtype, barriers) if shared_planes else None
    for tr in range(nty):
        for tc in range(ntx):
            t = shared if shared is not None else Tile(wav, rb, nb, dtype, barriers)
            qc = tc * ix - hq + np.arange(TX)
            cl = np.array([mirror(2 * c, w) >> 1 for c in qc])
            ch = np.array([mirror(2 * c + 1, w) >> 1 for c in qc])
            cell = CELL[wav]
            rm = mirror(2 * (tr * iy // cell * cell + cell // 2), h) >> 1
            c = dtype(np.rint(coef[rm, cl].sum() / TX))
            for wv in range(NW):
                for j in range(rb):
                    qr = tr * iy - hq + j * NW + wv
                    rl, rh = mirror(2 * qr, h) >> 1, mirror(2 * qr + 1, h) >> 1
                    t.q[wv, j, LL] = (coef[rl, cl] - c) / sll
                    t.q[wv, j, HL] = coef[rl, qw + ch]
                    t.q[wv, j, LH] = coef[qh + rh, cl]
                    t.q[wv, j, HH] = coef[qh + rh, qw + ch] / shh
            t.inverse()
            for wv in range(NW):
                for j in range(rb):
                    r = j * NW + wv
                    qr = tr * iy - hq + r
                    if r < hq or r >= NW * rb - hq or qr >= qh:
                        continue
                    for lane in range(hq, TX - hq):
                        cc = qc[lane]
                        if cc >= qw:
                            continue
                        px = 2 * cc
                        out[2 * qr, px] = t.q[wv, j, LL, lane] + c
                        if px + 1 < w:
                            out[2 * qr, px + 1] = t.q[wv, j, HL, lane] + c
                        if 2 * qr + 1 < h:
                            out[2 * qr + 1, px] = t.q[wv, j, LH, lane] + c
                            if px + 1 < w:
                                out[2 * qr + 1, px + 1] = t.q[wv, j, HH, lane] + c
    return out

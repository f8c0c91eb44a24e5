"""CPU walk of the marching restriction (restrict_march_kernel): the host's
plan and tile choice, every lane's loads (the pair of fine cells, the edge
cell of a 64-lane segment, the rows and planes of the march) and stores,
for the level shapes the tests and the benchmarked workloads use and every
tile; the lane shifts as the DPP wave shifts give them (lane i gets lane
i - 1's value, the first lane keeps its own; likewise upwards).  The values
the walk forms follow the kernel's arithmetic step by step and are compared
with the oracle's dense T (transposed); every coarse cell is written once.
The node-based kernel (lanes over the flattened coarse plane, a march of two
coarse planes per wave) is walked the same way against the node-based T."""
import numpy as np
import pytest

from oracle import multigrid as mg


def choose_tile(cnx, cny, cnz, groups, spanz, req):
    YR, ZR = (req >> 6, req & 63) if req else (2, 4)
    if not req and spanz:
        cells = cnx * cny * cnz
        if cells >= 128 ** 3:
            YR, ZR = 4, 8
        elif cells > 32 ** 3:
            YR, ZR = 2, 4
        else:
            YR, ZR = 2, 1
        if cny % (groups * YR) or cnz % ZR:
            YR, ZR = 2, 1
    if not spanz:
        ZR = 1
    return YR, ZR


def plan(fine, coarse, req=0):
    nz, ny, nx = fine
    cnz, cny, cnx = coarse
    if nx != 2 * cnx or ny != 2 * cny:
        return None
    spanz = nz > 1
    if (nz != 2 * cnz) if spanz else (cnz != 1):
        return None
    if cnx % 64 == 0:
        W, nseg = 64, cnx // 64
    elif 16 <= cnx < 64 and cnx & (cnx - 1) == 0:
        W, nseg = cnx, 1
    else:
        return None
    groups = 64 // W
    YR, ZR = choose_tile(cnx, cny, cnz if spanz else 1, groups, spanz, req)
    if cny % (groups * YR) or (spanz and cnz % ZR):
        return None
    assert nz * ny * nx * 4 < 2 ** 31
    return dict(W=W, wshift=W.bit_length() - 1, groups=groups, nseg=nseg, YR=YR, ZR=ZR,
                nyc=cny // (groups * YR), nzc=cnz // ZR if spanz else 1, spanz=spanz)


def t_entry(r, J, n):
    if r == 0:
        return 1.25 if J == 0 else (-0.25 if J == 1 else 0.0)
    if r == 2 * n - 1:
        return 1.25 if J == n - 1 else (-0.25 if J == n - 2 else 0.0)
    K = r >> 1
    nb = K + 1 if r & 1 else K - 1
    return 0.75 if J == K else (0.25 if J == nb else 0.0)


def taps6(J, n):
    s = min(max(2 * J - 1, 0), 2 * n - 4)
    idx = [s + k for k in range(4)] + [0, 2 * n - 1]
    w = [t_entry(s + k, J, n) for k in range(4)]
    w += [t_entry(0, J, n) if s > 0 else 0.0, t_entry(2 * n - 1, J, n) if s + 3 < 2 * n - 1 else 0.0]
    return idx, w


def row_of(k, Y0, ny, YR):
    if k == 0:
        return 2 * Y0 - 1 if Y0 > 0 else 0
    if k <= 2 * YR:
        return 2 * Y0 + k - 1
    return 2 * (Y0 + YR) if 2 * (Y0 + YR) < ny else ny - 1


def prev(v):
    out = v.copy()
    out[1:] = v[:-1]
    return out


def nxt(v):
    out = v.copy()
    out[:-1] = v[1:]
    return out


class Walk:
    def __init__(self, g, P):
        self.g, self.P = g, P
        self.nz, self.ny, self.nx = g.shape

    def load_row(self, z, row, loff_cells, ed):
        assert 0 <= z < self.nz and 0 <= row < self.ny
        assert np.all((loff_cells >= 0) & (loff_cells + 1 < self.nx))
        r = self.g[z, row]
        a, b = r[loff_cells], r[loff_cells + 1]
        e = None
        if self.P["nseg"] > 1:
            ei = loff_cells + ed
            assert np.all((ei >= 0) & (ei < self.nx))
            e = r[ei]
        return a, b, e

    def x_restrict(self, a, b, e, gl, cx, cnx):
        W = self.P["W"]
        left, right, e0, e1 = prev(b), nxt(a), prev(a), nxt(b)
        if e is not None:
            left = np.where(gl == 0, e, left)
            right = np.where(gl == W - 1, e, right)
        x = np.where(cx == 0, 1.25, 0.75) * a + np.where(cx == cnx - 1, 1.25, 0.75) * b
        x = x + np.where(cx > 0, 0.25 * left, 0.0)
        x = x + np.where(cx < cnx - 1, 0.25 * right, 0.0)
        x = x - np.where(cx == 1, 0.25 * e0, 0.0)
        x = x - np.where(cx == cnx - 2, 0.25 * e1, 0.0)
        return x

    def y_restrict(self, z, Y0, loff, ed, gl, cx, cnx):
        YR, ny = self.P["YR"], self.ny
        cny = ny >> 1
        Pj = [np.zeros(64) for _ in range(YR)]
        for k in range(2 * YR + 2):
            # every lane of a row group shares Y0; lanes of different groups differ
            rows = np.array([row_of(k, int(y), ny, YR) for y in Y0])
            a = np.empty(64)
            b = np.empty(64)
            e = np.empty(64) if self.P["nseg"] > 1 else None
            for r in np.unique(rows):
                m = rows == r
                aa, bb, ee = self.load_row(z, r, loff[m], ed[m])
                a[m], b[m] = aa, bb
                if e is not None:
                    e[m] = ee
            x = self.x_restrict(a, b, e, gl, cx, cnx)
            for lane in range(64):
                y0 = int(Y0[lane])
                if k == 0:
                    if y0 > 0:
                        Pj[0][lane] += 0.25 * x[lane]
                elif k <= 2 * YR:
                    j = (k - 1) >> 1
                    if k & 1:
                        end = y0 + j == 0
                        Pj[j][lane] += (1.25 if end else 0.75) * x[lane]
                        if end:
                            if j + 1 < YR:
                                Pj[j + 1][lane] -= 0.25 * x[lane]
                        elif j >= 1:
                            Pj[j - 1][lane] += 0.25 * x[lane]
                    else:
                        end = y0 + j == cny - 1
                        Pj[j][lane] += (1.25 if end else 0.75) * x[lane]
                        if end:
                            if j >= 1:
                                Pj[j - 1][lane] -= 0.25 * x[lane]
                        elif j + 1 < YR:
                            Pj[j + 1][lane] += 0.25 * x[lane]
                else:
                    if y0 + YR < cny:
                        Pj[YR - 1][lane] += 0.25 * x[lane]
        return Pj

    def run(self, coarse):
        P = self.P
        cnz, cny, cnx = coarse
        out = np.full(coarse, np.nan)
        writes = np.zeros(coarse, dtype=np.int64)
        lane = np.arange(64)
        n_tasks = P["nseg"] * P["nyc"] * P["nzc"]
        YR, ZR = P["YR"], P["ZR"]

        def emit(Zc, Y0, cx, vals):
            for j in range(YR):
                y = Y0 + j
                assert np.all((y >= 0) & (y < cny)) and np.all((cx >= 0) & (cx < cnx))
                out[Zc, y, cx] = vals[j]
                np.add.at(writes, (np.full(64, Zc), y, cx), 1)

        for task in range(n_tasks):
            t = task
            yc = t % P["nyc"]; t //= P["nyc"]
            zc = t % P["nzc"]; t //= P["nzc"]
            seg = t % P["nseg"]
            grp, gl = lane >> P["wshift"], lane & (P["W"] - 1)
            cx = seg * 64 + gl
            Y0 = (yc * P["groups"] + grp) * YR
            seg_on = P["nseg"] > 1
            ed = np.where(seg_on & (gl == 0) & (cx > 0), -1,
                          np.where(seg_on & (gl == P["W"] - 1) & (cx < cnx - 1), 2, 0))
            loff = 2 * cx
            if not P["spanz"]:
                emit(0, Y0, cx, self.y_restrict(0, Y0, loff, ed, gl, cx, cnx))
                continue
            Z0 = zc * ZR
            if ZR == 1:
                iz, wz = taps6(Z0, cnz)
                acc = [np.zeros(64) for _ in range(YR)]
                for zz, w in zip(iz, wz):
                    if w != 0.0:
                        Pz = self.y_restrict(zz, Y0, loff, ed, gl, cx, cnx)
                        for j in range(YR):
                            acc[j] += w * Pz[j]
                emit(Z0, Y0, cx, acc)
                continue
            Ap = [np.zeros(64) for _ in range(YR)]
            Ac = [np.zeros(64) for _ in range(YR)]
            An = [np.zeros(64) for _ in range(YR)]
            Jbeg, Jend = max(Z0 - 1, 0), min(Z0 + ZR, cnz - 1)
            nz = self.nz
            for J in range(Jbeg, Jend + 1):
                za, zb = 2 * J, 2 * J + 1
                emit_now = Z0 <= J - 1 < Z0 + ZR
                needA = not (J == Z0 - 1 and za != 0)
                needB = not (J == Z0 + ZR and zb != nz - 1)
                if needA:
                    Pa = self.y_restrict(za, Y0, loff, ed, gl, cx, cnx)
                    wa = 1.25 if za == 0 else 0.75
                    for j in range(YR):
                        Ac[j] += wa * Pa[j]
                        if za == 0:
                            An[j] -= 0.25 * Pa[j]
                        else:
                            Ap[j] += 0.25 * Pa[j]
                if needB:
                    Pb = self.y_restrict(zb, Y0, loff, ed, gl, cx, cnx)
                    last = zb == nz - 1
                    wb = 1.25 if last else 0.75
                    for j in range(YR):
                        Ac[j] += wb * Pb[j]
                        if last:
                            Ap[j] -= 0.25 * Pb[j]
                        else:
                            An[j] += 0.25 * Pb[j]
                if emit_now:
                    emit(J - 1, Y0, cx, Ap)
                Ap, Ac, An = Ac, An, [np.zeros(64) for _ in range(YR)]
            if Jend == cnz - 1 and Z0 <= cnz - 1 < Z0 + ZR:
                emit(cnz - 1, Y0, cx, Ap)
        assert np.all(writes == 1), np.unique(writes, return_counts=True)
        return out


def oracle_restrict(g, coarse):
    out = g
    for ax in range(3):
        if g.shape[ax] == 1:
            continue
        T = mg.cell_T_matrix(coarse[ax])
        out = np.moveaxis(np.tensordot(T.T, np.moveaxis(out, ax, 0), axes=1), 0, ax)
    return out


CASES = [((128, 128, 128), 0), ((64, 64, 64), 0), ((32, 32, 32), 0), ((256, 256, 256), 0),
         ((16, 128, 128), 0), ((8, 64, 64), 0), ((1, 128, 128), 0), ((1, 64, 64), 0),
         ((1, 256, 256), 0), ((32, 64, 128), 0), ((64, 32, 64), 0)]
TILES = [(2, 1), (2, 2), (2, 4), (2, 8), (4, 1), (4, 2), (4, 4), (4, 8), (4, 16), (8, 4), (8, 8)]
CASES += [((32, 64, 128), 64 * r + z) for r, z in TILES]


@pytest.mark.parametrize("fine,req", CASES)
def test_march_walk(fine, req):
    coarse = tuple(n // 2 if n > 1 else 1 for n in fine)
    P = plan(fine, coarse, req)
    assert P is not None, (fine, req)
    if req:
        assert (P["YR"], P["ZR"]) == (req >> 6, req & 63)
    g = np.random.default_rng(sum(fine) + req).standard_normal(fine)
    got = Walk(g, P).run(coarse)
    want = oracle_restrict(g, coarse)
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-12 * np.abs(want).max())


def test_the_benchmarked_levels_take_their_tiles():
    """128^3 -> 64^3 marches (2, 4), 256^3 -> 128^3 (4, 8) in 64-lane
    segments, 32^3 and below one plane per wave."""
    p = plan((128,) * 3, (64,) * 3)
    assert (p["YR"], p["ZR"], p["W"], p["nseg"]) == (2, 4, 64, 1)
    p = plan((256,) * 3, (128,) * 3)
    assert (p["YR"], p["ZR"], p["W"], p["nseg"]) == (4, 8, 64, 2)
    p = plan((64,) * 3, (32,) * 3)
    assert (p["YR"], p["ZR"], p["W"], p["groups"]) == (2, 1, 32, 2)


# ---------------------------------------------------------------- node-based
def node_plan(fine, coarse):
    nz, ny, nx = fine
    cnz, cny, cnx = coarse
    if nx != 2 * cnx - 1 or ny != 2 * cny - 1 or cnx < 2 or cny < 2:
        return None
    spanz = nz > 1
    if (nz != 2 * cnz - 1) if spanz else (cnz != 1):
        return None
    plane = cny * cnx
    tasks_plane = -(-plane // 64)
    zr = 2 if spanz else 1
    if spanz and 5 * ((cnz + 1) // 2) * tasks_plane < 2048:  # five fields, one instance
        zr = 1
    return dict(lanes=plane, tasks_plane=-(-plane // 64), zr=zr, nzc=-(-cnz // zr) if spanz else 1,
                spanz=spanz)


def node_walk(g, coarse, P):
    """The node kernel's lanes over the flattened coarse plane, its loads,
    shifts, z march and stores, with bounds checks."""
    nfz, nfy, nfx = g.shape
    ncz, ncy, ncx = coarse
    out = np.full(coarse, np.nan)
    writes = np.zeros(coarse, dtype=np.int64)
    lane = np.arange(64)
    for zc in range(P["nzc"]):
        for tp in range(P["tasks_plane"]):
            qn = tp * 64 + lane
            on = qn < P["lanes"]
            qc = np.where(on, qn, P["lanes"] - 1)
            Y, J = qc // ncx, qc % ncx
            has_b = 2 * J + 1 < nfx
            self_left = (lane == 0) & (J > 0)
            rows, wy = [], []
            for k in range(3):
                r = 2 * Y - 1 + k
                rows.append(np.clip(r, 0, nfy - 1))
                wy.append(np.where((r < 0) | (r >= nfy), 0.0, 1.0 if k == 1 else 0.5))

            def plane_value(z):
                assert 0 <= z < nfz
                acc = np.zeros(64)
                for k in range(3):
                    assert np.all((rows[k] >= 0) & (rows[k] < nfy))
                    assert np.all(2 * J < nfx)
                    a = g[z, rows[k], 2 * J]
                    bb = np.where(has_b, g[z, rows[k], np.minimum(2 * J + 1, nfx - 1)], 0.0)
                    assert np.all(2 * J[self_left] - 1 >= 0)
                    e = np.where(self_left, g[z, rows[k], np.maximum(2 * J - 1, 0)], 0.0)
                    left = prev(bb)
                    left = np.where(self_left, e, left)
                    left = np.where(J == 0, 0.0, left)
                    acc += wy[k] * (a + 0.5 * left + 0.5 * bb)
                return acc

            def finish(Jz, val):
                assert 0 <= Jz < ncz
                out[Jz, Y[on], J[on]] = val[on]
                np.add.at(writes, (np.full(on.sum(), Jz), Y[on], J[on]), 1)

            if not P["spanz"]:
                finish(0, plane_value(0))
                continue
            Z0 = zc * P["zr"]
            Z1 = min(Z0 + P["zr"], ncz)
            odd = plane_value(2 * Z0 - 1) if Z0 > 0 else np.zeros(64)
            for Jz in range(Z0, Z1):
                even = plane_value(2 * Jz)
                nx_ = plane_value(2 * Jz + 1) if 2 * Jz + 1 < nfz else np.zeros(64)
                finish(Jz, 0.5 * odd + even + 0.5 * nx_)
                odd = nx_
    assert np.all(writes == 1)
    return out


NODE_CASES = [(65, 65, 129), (33, 33, 65), (17, 17, 33), (1, 65, 65), (1, 33, 33), (1, 129, 129),
              (9, 17, 33), (5, 9, 17), (3, 5, 9)]


@pytest.mark.parametrize("fine", NODE_CASES)
def test_node_march_walk(fine):
    coarse = tuple(1 if n == 1 else (n - 1) // 2 + 1 for n in fine)
    P = node_plan(fine, coarse)
    assert P is not None
    g = np.random.default_rng(sum(fine)).standard_normal(fine)
    got = node_walk(g, coarse, P)
    want = g
    for ax in range(3):
        if fine[ax] == 1:
            continue
        T = mg.node_T_matrix(coarse[ax] - 1)
        want = np.moveaxis(np.tensordot(T.T, np.moveaxis(want, ax, 0), axes=1), 0, ax)
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-12 * np.abs(want).max())

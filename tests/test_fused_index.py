"""Index walk of the fused channel-flow kernel on the host: the tile mapping,
the thread roles, every LDS slot and every 32-bit global byte offset the
kernel forms, for every block, thread and plane of the problem sizes the GPU
tests and the benchmark use.  The formulas restate the kernel's index
arithmetic (tiles of 32 x 16 owned cells with a 2-cell halo, 768 threads,
z-chunks of 16/8/4/2 planes, the level-1 window of 20 x 12 coarse cells, the
optional z sums of the gradient); a slot or offset outside its array, a cell
owned twice or not at all, or an offset past 2^32 fails here, on the CPU."""
import numpy as np
import pytest

NSO_X, NSO_Y = 32, 16
NST_X, NST_Y = NSO_X + 4, NSO_Y + 4
NS_MAIN = NSO_X * NST_Y
NS_HALO = 4 * NST_Y
NS_THREADS = NS_MAIN + (NS_HALO + 63) // 64 * 64
NS_XCD, CUS = 8, 256
NCT_X, NCT_Y = NST_X // 2 + 2, NST_Y // 2 + 2
NF_MAX = 5


def tiles(nz, ny, nx, batch):
    ntx = -(-nx // NSO_X)
    nty = -(-ny // NSO_Y)
    xy = ntx * nty * batch
    tz = 32
    while tz > 2 and xy * (-(-nz // tz)) < CUS:
        tz //= 2
    return tz, -(-nz // tz), ntx, nty


def threads():
    tid = np.arange(NS_THREADS)
    X = np.zeros_like(tid)
    Y = np.zeros_like(tid)
    active = np.ones(NS_THREADS, bool)
    main = tid < NS_MAIN
    X[main] = 2 + tid[main] % NSO_X
    Y[main] = tid[main] // NSO_X
    halo = (tid >= NS_MAIN) & (tid < NS_MAIN + NS_HALO)
    h = tid[halo] - NS_MAIN
    c = h // NST_Y
    X[halo] = np.where(c < 2, c, NSO_X + c)
    Y[halo] = h % NST_Y
    active[tid >= NS_MAIN + NS_HALO] = False
    return tid, X, Y, active


def prolong_taps(i, n):
    """Cell-based T taps of fine cell i (of 2n): parent and neighbour."""
    J = i >> 1
    nb = np.where(i & 1, J + 1, J - 1)
    lo = nb < 0
    hi = nb >= n
    j1 = np.where(lo, J + 1, np.where(hi, J - 1, nb))
    return J, j1


CASES = [((24, 36, 60), 1, 3), ((16, 28, 24), 1, 3), ((64, 16, 32), 1, 4), ((8, 8, 8), 1, 1),
         ((16, 16, 24), 1, 3), ((8, 16, 24), 1, 3), ((16, 24, 32), 2, 3), ((40, 12, 20), 4, 3),
         ((40, 12, 20), 26, 3), ((40, 12, 20), 52, 3), ((40, 12, 20), 86, 3), ((40, 12, 20), 130, 3),
         ((16, 16, 32), 1, 3),
         ((32, 32, 64), 1, 4), ((64, 64, 64), 1, 5), ((128, 128, 128), 1, 6),
         ((16, 128, 128), 1, 4), ((256, 256, 256), 1, 7), ((8, 8, 16), 1, 3),
         ((4, 4, 4), 1, 1), ((4, 4, 4), 1, 2), ((4, 8, 12), 1, 2)]


@pytest.mark.parametrize("dims,batch,L", CASES)
@pytest.mark.parametrize("nf", [5, 4])
@pytest.mark.parametrize("elem", [4, 8])
def test_fused_kernel_indices(dims, batch, L, nf, elem):
    """Element size 8 is the FP64 build of the same source (switched off in
    the library): its byte offsets stay in bounds too at the sizes where it
    was tested, so no out-of-range access explains its wrong results."""
    nz, ny, nx = dims
    if elem == 8 and nf * nz * ny * nx * elem >= 2 ** 32:
        pytest.skip("beyond the 32-bit offsets an FP64 field set would need")
    tz, nzt, ntx, nty = tiles(nz, ny, nx, batch)
    ntiles = nzt * ntx * nty
    tpx = -(-ntiles // NS_XCD)
    # ---- block -> (instance, tile): every pair exactly once
    blocks = np.arange(NS_XCD * tpx * batch)
    per_inst = NS_XCD * tpx
    inst = blocks // per_inst
    bl = blocks - inst * per_inst
    tile = (bl % NS_XCD) * tpx + bl // NS_XCD
    ok = tile < ntiles
    pairs = inst[ok] * ntiles + tile[ok]
    assert np.array_equal(np.sort(pairs), np.arange(batch * ntiles))
    # ---- thread roles cover the 36 x 20 tile once
    tid, X, Y, active = threads()
    pos = Y[active] * NST_X + X[active]
    assert np.array_equal(np.sort(pos), np.arange(NST_X * NST_Y))
    fsize = nz * ny * nx
    plane = nx * ny
    assert nf * fsize * elem < 2 ** 32         # the host's 32-bit offset condition
    owned = np.zeros(batch * nzt * ny * nx, np.int64)
    for t in range(ntiles):
        bx, by, bz = t % ntx, (t // ntx) % nty, t // (ntx * nty)
        ox, oy = bx * NSO_X - 2, by * NSO_Y - 2
        x, y = ox + X, oy + Y
        z0, z1 = bz * tz, min(bz * tz + tz, nz)
        in_xy = active & (x >= 0) & (x < nx) & (y >= 0) & (y < ny)
        seed = in_xy & (X >= 1) & (X <= NST_X - 2) & (Y >= 1) & (Y <= NST_Y - 2)
        own = in_xy & (X >= 2) & (X <= NST_X - 3) & (Y >= 2) & (Y <= NST_Y - 3)
        # LDS: staged plane, wall slots across the grid's walls, stencil and gather reads
        for cond, dx, dy in ((seed & (x == 0), -1, 0), (seed & (x == nx - 1), 1, 0),
                             (seed & (y == 0), 0, -1), (seed & (y == ny - 1), 0, 1)):
            xs, ys = X[cond] + dx, Y[cond] + dy
            assert np.all((xs >= 0) & (xs < NST_X) & (ys >= 0) & (ys < NST_Y))
        for m in (seed, own):
            for dx, dy in ((-1, 0), (1, 0), (0, -1), (0, 1)):
                xs, ys = X[m] + dx, Y[m] + dy
                assert np.all((xs >= 0) & (xs < NST_X) & (ys >= 0) & (ys < NST_Y))
        # ownership of the chunk's columns
        col = y * nx + x
        owned_idx = bz * plane + col[own]
        np.add.at(owned, owned_idx, 1)  # instance 0's tiles; the others are the same
        # global byte offsets: column in the last field plus the farthest plane
        fo = ((nf - 1) * fsize + np.where(in_xy, col, 0)) * elem
        planes = [z for z in range(z0 - 2, z1 + 2) if 0 <= z < nz]
        assert np.all(fo + max(planes) * plane * elem < nf * fsize * elem)
        assert np.all(fo + max(planes) * plane * elem < 2 ** 32)
        if L > 1:
            nc = (nz // 2, ny // 2, nx // 2)
            cxb, cyb = (ox >> 1) - 1, (oy >> 1) - 1
            jx = prolong_taps(x[in_xy], nc[2])
            jy = prolong_taps(y[in_xy], nc[1])
            for j in jx:
                assert np.all((j - cxb >= 0) & (j - cxb < NCT_X)), "x window"
                assert np.all((j >= 0) & (j < nc[2]))
            for j in jy:
                assert np.all((j - cyb >= 0) & (j - cyb < NCT_Y)), "y window"
                assert np.all((j >= 0) & (j < nc[1]))
            # coarse planes the march reads: kbase(z) and kbase(z) + 1 of every plane
            zs = np.array(planes)
            kb = np.where(zs == 0, 0, np.where(zs == nz - 1, nc[0] - 2, np.where(zs & 1, zs // 2, zs // 2 - 1)))
            assert np.all((kb >= 0) & (kb + 1 < nc[0]))
            # the window values the threads move: offsets inside level 1
            e = np.concatenate([tid, tid + NS_THREADS])
            e = e[e < nf * NCT_X * NCT_Y]
            assert nf * NCT_X * NCT_Y <= 2 * NS_THREADS
            f, rem = e // (NCT_X * NCT_Y), e % (NCT_X * NCT_Y)
            cy, cx = cyb + rem // NCT_X, cxb + rem % NCT_X
            cin = (cy >= 0) & (cy < nc[1]) & (cx >= 0) & (cx < nc[2])
            csize = nc[0] * nc[1] * nc[2]
            co = (f[cin] * csize + cy[cin] * nc[2] + cx[cin]) * elem
            assert np.all(co + (nc[0] - 1) * nc[1] * nc[2] * elem < nf * csize * elem)
            # z sums of the gradient (optional path): slots and offsets
            hz, kz0 = tz // 2, z0 // 2 - 1
            nkz = hz + 2
            for q in range(z0, z1):
                for K in prolong_taps(np.array([q]), nc[0]):
                    assert 0 <= int(K[0]) - kz0 < nkz
            zmax = ((nkz - 1) * plane + (nf - 1) * nkz * plane + col[own]) * elem
            assert np.all(zmax < nf * nkz * plane * elem) and np.all(zmax < 2 ** 32)
    # every cell of every chunk owned exactly once
    assert np.all(owned[:nzt * plane] == 1)


def test_measurement_positions_in_tile():
    """A measurement's position in its tile (halo included) is inside the staged plane."""
    for nz, ny, nx in ((24, 36, 60), (128, 128, 128), (40, 12, 20)):
        idx = np.arange(nz * ny * nx)
        lx = idx % nx % NSO_X + 2
        ly = idx // nx % ny % NSO_Y + 2
        assert np.all((lx >= 2) & (lx < NST_X - 2) & (ly >= 2) & (ly < NST_Y - 2))


NODE_CASES = [((16, 16, 24), 1, 3), ((8, 12, 20), 1, 2), ((8, 16, 24), 1, 3), ((16, 16, 32), 1, 3),
              ((64, 64, 128), 1, 6), ((32, 32, 64), 1, 4), ((8, 8, 16), 1, 3)]


@pytest.mark.parametrize("dims,batch,L", NODE_CASES)
def test_fused_kernel_indices_node(dims, batch, L):
    """Node-based values: the kernel marches over the interior nodes (cells
    = nodes 1 .. N - 1 per axis); fields are stored with the boundary nodes
    (N + 1 per axis); the level-1 window holds the coarse nodes of the node
    taps (even fine node: one coarse node, odd: the two around it)."""
    nf = 5
    nz, ny, nx = (d - 1 for d in dims)            # interior nodes
    tz, nzt, ntx, nty = tiles(nz, ny, nx, batch)
    tid, X, Y, active = threads()
    sx, sy, sz = nx + 2, ny + 2, nz + 2
    fsize, plane = sx * sy * sz, sx * sy
    owned = np.zeros(nzt * plane, np.int64)
    for t in range(nzt * ntx * nty):
        bx, by, bz = t % ntx, (t // ntx) % nty, t // (ntx * nty)
        ox, oy = bx * NSO_X - 2, by * NSO_Y - 2
        x, y = ox + X, oy + Y
        z0, z1 = bz * tz, min(bz * tz + tz, nz)
        in_xy = active & (x >= 0) & (x < nx) & (y >= 0) & (y < ny)
        own = in_xy & (X >= 2) & (X <= NST_X - 3) & (Y >= 2) & (Y <= NST_Y - 3)
        col = (y + 1) * sx + (x + 1)
        np.add.at(owned, bz * plane + col[own], 1)
        planes = [z for z in range(z0 - 2, z1 + 2) if 0 <= z < nz]
        fo = ((nf - 1) * fsize + np.where(in_xy, col, 0)) * 4
        assert np.all(fo + (max(planes) + 1) * plane * 4 < nf * fsize * 4)
        if L > 1:
            nc = tuple(d // 2 + 1 for d in dims)   # coarse nodes per axis
            cxb, cyb = (ox >> 1) - 1, (oy >> 1) - 1
            for v, cb, w, n in ((x[in_xy] + 1, cxb, NCT_X, nc[2]), (y[in_xy] + 1, cyb, NCT_Y, nc[1])):
                for J in (v >> 1, (v >> 1) + (v & 1)):
                    assert np.all((J - cb >= 0) & (J - cb < w))
                    assert np.all((J >= 0) & (J < n))
            zs = np.array(planes)
            kb = np.minimum((zs + 1) >> 1, nc[0] - 2)
            assert np.all((kb >= 0) & (kb + 1 < nc[0]))
            # the coarse planes of each fine node plane are the resident pair
            n = zs + 1
            assert np.all(((n & 1) == 1) | (n // 2 == kb) | (n // 2 == kb + 1))
            assert np.all(((n & 1) == 0) | ((n >> 1) == kb))
    # every interior node of every chunk owned once, no boundary node owned
    inner = np.zeros((sy, sx), bool)
    inner[1:-1, 1:-1] = True
    for bz in range(nzt):
        got = owned[bz * plane:(bz + 1) * plane].reshape(sy, sx)
        assert np.all(got[inner] == 1) and np.all(got[~inner] == 0)


@pytest.mark.parametrize("dims,batch,L", NODE_CASES)
def test_node_boundary_regions(dims, batch, L):
    """Node-based: the blocks' regions (their owned interior nodes plus the
    boundary nodes beyond them at the grid's ends) partition the node grid,
    and the faces each block walks (first face wins at edges and corners)
    give every boundary node exactly once and no interior node."""
    nz, ny, nx = (d - 1 for d in dims)
    tz, nzt, ntx, nty = tiles(nz, ny, nx, batch)
    last = (nz + 1, ny + 1, nx + 1)
    count = np.zeros(tuple(v + 1 for v in last), np.int64)
    for t in range(nzt * ntx * nty):
        bx, by, bz = t % ntx, (t // ntx) % nty, t // (ntx * nty)
        z0, z1 = bz * tz, min(bz * tz + tz, nz)
        lo = (0 if bz == 0 else z0 + 1, 0 if by == 0 else by * NSO_Y + 1, 0 if bx == 0 else bx * NSO_X + 1)
        hi = (last[0] if bz == nzt - 1 else z1, last[1] if by == nty - 1 else min(by * NSO_Y + NSO_Y, ny),
              last[2] if bx == ntx - 1 else min(bx * NSO_X + NSO_X, nx))
        for a in range(3):
            for side in range(2):
                fixed = last[a] if side else 0
                if (hi[a] if side else lo[a]) != fixed:
                    continue
                b1, b2 = (a + 1) % 3, (a + 2) % 3
                for e in range((hi[b1] - lo[b1] + 1) * (hi[b2] - lo[b2] + 1)):
                    c = [0, 0, 0]
                    c[a] = fixed
                    c[b1] = lo[b1] + e // (hi[b2] - lo[b2] + 1)
                    c[b2] = lo[b2] + e % (hi[b2] - lo[b2] + 1)
                    if any(c[a2] in (0, last[a2]) for a2 in range(a)):
                        continue
                    count[tuple(c)] += 1
    boundary = np.ones(count.shape, bool)
    boundary[1:-1, 1:-1, 1:-1] = False
    assert np.all(count[boundary] == 1) and np.all(count[~boundary] == 0)

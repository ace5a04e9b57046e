"""Host checks of the kernels' thread-to-element maps (CPU only).

The index arithmetic of the work distributions that are not a plain
consecutive mapping is restated here in numpy and checked on the workload's
and the tests' shapes: every element is reached exactly once, every access
stays inside its array, and each wave holds what its kernel assumes (one
shift per wave, lane 0 at the wave's smallest element).  These are the
invariants the kernels rely on for in-bounds access; a change to the
kernels' maps must keep them (and this restatement must follow).

* the gathered y-sweep map of k_position (FP32 storage): waves of 8 whole
  uz-lines of one u_y from 8 u_x rows, work-groups of a unit eight apart so
  that they share an XCD;
* the slab walk of k_kick_yz64 (64^3 blocks): persistent work-groups over
  (cell, slab) pairs;
* the 4-value slots of the fused kick's block (k_kick), the 64-cell uz tiles
  (k_vel_uz_tiles) and the slabs (k_kick_yz64): consecutive threads take
  consecutive 16-byte groups, and each lands in its padded LDS line;
* the in-place rotation of a periodic 64-value line by the integer part of
  its shift (translate_line: three reversals, in either walk direction);
* the y-sweep adjoint's permutation (k_position_adj): one u_y per wave.
"""
import numpy as np
import pytest


def gathered_y_map(nx, nz, nux, nuy, nuz, V=4):
    """(global element, shift index) of every thread, in thread order."""
    Nu = nux * nuy * nuz
    O, I = nx, nz * Nu
    IV = I // V
    R = 64 * V // nuz
    Q = nuy // 4
    nblocks = O * IV // 256
    b = np.arange(nblocks)[:, None]
    tx = np.arange(256)[None, :]
    sup = b // (8 * Q)
    rem = b - sup * 8 * Q
    unit = sup * 8 + rem % 8
    jy = (rem // 8) * 4 + (tx >> 6)
    lane = tx & 63
    ngx = nux // R
    upr = (I // Nu) * ngx
    o = unit // upr
    ur = unit - o * upr
    blk = ur // ngx
    jxg = ur - blk * ngx
    G = nuz // V
    rr = lane // G
    k0 = blk * Nu + (jxg * R * nuy + jy) * nuz
    k = k0 + rr * nuy * nuz + (lane - rr * G) * V
    return (o * I + k).ravel(), (((k % Nu) // nuz) % nuy).ravel(), k.ravel(), k0.ravel()


def gathered_y_applies(nx, nz, nux, nuy, nuz, V=4):
    """The host's conditions (make_pos_args) for the gathered map."""
    I = nz * nux * nuy * nuz
    if (64 * V) % nuz or (I // V) % 256 or nuy % 4:
        return False
    R = 64 * V // nuz
    units = nx * nz * (nux // R) if R > 0 else 0
    return R > 1 and nux % R == 0 and (nuz // V) * R == 64 and units % 8 == 0


@pytest.mark.parametrize("shape", [(64, 64, 32, 32, 32), (16, 16, 16, 16, 16), (8, 5, 32, 32, 32),
                                   (4, 4, 64, 64, 64), (2, 2, 64, 64, 64)])
def test_gathered_y_map(shape):
    nx, nz, nux, nuy, nuz = shape
    V = 4
    if not gathered_y_applies(nx, nz, nux, nuy, nuz, V):
        pytest.skip("the host does not take the gathered map for this shape")
    g, jl, k, k0 = gathered_y_map(nx, nz, nux, nuy, nuz, V)
    total = nx * nz * nux * nuy * nuz
    assert g.min() == 0 and g.max() == total - V
    assert np.all(g % V == 0)
    assert len(np.unique(g)) == total // V               # each group of V once
    waves = jl.reshape(-1, 64)
    assert np.all(waves == waves[:, :1])                 # one u_y (shift) per wave
    kw, k0w = k.reshape(-1, 64), k0.reshape(-1, 64)
    assert np.all(kw.min(axis=1) == kw[:, 0]) and np.all(k0w[:, 0] == kw[:, 0])
    # a unit (row o, spatial cell, group of R u_x rows) read back from the
    # elements each work-group touches: nu_y / 4 work-groups, all with the
    # same block index mod 8 (one XCD under round-robin dispatch)
    Nu, R = nux * nuy * nuz, 64 * V // nuz
    gw = g.reshape(-1, 256)
    jx = (gw % Nu) // (nuy * nuz)
    units = (gw // Nu) * (nux // R) + jx // R          # (o, cell) row-major, then u_x group
    assert np.all(units == units[:, :1])              # a work-group stays in one unit
    u = units[:, 0]
    _, counts = np.unique(u, return_counts=True)
    assert np.all(counts == nuy // 4)
    assert len(np.unique(u * 8 + np.arange(len(u)) % 8)) == len(counts)


def slab_walk(b, G, C, nslab=8):
    """(cell, slab) pairs of persistent work-group b of G over C cells."""
    out, cell = [], b
    if cell >= C:
        return out
    slab = 0
    ncl, nsl = (cell, 1) if nslab > 1 else (cell + G, 0)
    while True:
        out.append((cell, slab))
        if ncl >= C:
            break
        cell, slab = ncl, nsl
        nsl, ncl = slab + 1, cell
        if nsl == nslab:
            nsl, ncl = 0, cell + G
    return out


@pytest.mark.parametrize("G,C", [(256, 32768), (256, 64), (7, 50), (1, 3), (300, 256)])
def test_slab_walk_covers_each_slab_once(G, C):
    seen = []
    for b in range(G):
        walk = slab_walk(b, G, C)
        # a work-group's slabs of one cell come in order and end with slab 7
        for (c0, s0), (c1, s1) in zip(walk, walk[1:]):
            assert (c1 == c0 and s1 == s0 + 1) or (s0 == 7 and s1 == 0 and c1 == c0 + G)
        seen += walk
    assert sorted(seen) == [(c, s) for c in range(C) for s in range(8)]


@pytest.mark.parametrize("nthreads,nvalues,nu", [(1024, 32 ** 3, 32),   # k_kick block
                                                 (256, 16 ** 3, 16),    # k_kick, 16^3 block
                                                 (256, 256 * 64, 64),   # k_vel_uz_tiles tile
                                                 (512, 8 * 64 * 64, 64)])  # k_kick_yz64 slab
def test_slots_fill_the_padded_lds_once(nthreads, nvalues, nu):
    ns = nvalues // (nthreads * 4)
    assert ns * nthreads * 4 == nvalues
    s = np.arange(ns)[:, None]
    t = np.arange(nthreads)[None, :]
    e = (s * nthreads + t) * 4                           # first value of each slot
    vals = (e[..., None] + np.arange(4)).ravel()
    assert np.array_equal(np.sort(vals), np.arange(nvalues))
    # consecutive threads take consecutive 16-byte groups (coalesced)
    assert np.all(np.diff(e, axis=1) == 4)
    # LDS position: line e // nu padded to nu + 1, offset e % nu; a group of
    # four never crosses a line, and positions are distinct and in range
    line, off = e // nu, e % nu
    assert np.all(off + 3 < nu)
    pos = ((line * (nu + 1) + off)[..., None] + np.arange(4)).ravel()
    assert len(np.unique(pos)) == nvalues
    assert pos.max() < (nvalues // nu) * (nu + 1)


def rotate_by_reversals(line, N, neg):
    """translate_line's periodic rotation of a 64-value line in place: frame
    position p at index (M-1-p if neg else p); reverse all positions, then
    0..N-1 and N..M-1."""
    M = len(line)
    x = list(line)
    at = (lambda p: M - 1 - p) if neg else (lambda p: p)

    def rev(lo, hi):
        i, j = lo, hi - 1
        while i < j:
            x[at(i)], x[at(j)] = x[at(j)], x[at(i)]
            i, j = i + 1, j - 1
    rev(0, M)
    rev(0, N)
    rev(N, M)
    return np.array(x)


@pytest.mark.parametrize("neg", [False, True])
def test_periodic_rotation_in_place(neg):
    # out_{p+N mod M} = y_p in frame positions; the frame runs against the
    # index for lines whose upwind direction is -u
    M = 64
    y = np.arange(M) * 1.0 + 0.5
    for N in range(1, M):
        got = rotate_by_reversals(y, N, neg)
        want = np.roll(y, -N if neg else N)
        assert np.array_equal(got, want), N


def adjoint_y_map(nz, nux, nuy, nuz):
    """k_position_adj's element of thread k of a row for y sweeps (pst = nu_z)."""
    I = nz * nux * nuy * nuz
    k = np.arange(I)
    G = 64 * nuy
    l = k & 63
    rr = l // nuz
    return (k // G) * G + (rr * nuy + (k % G) // 64) * nuz + (l - rr * nuz)


@pytest.mark.parametrize("nz,nux,nuy,nuz", [(32, 16, 16, 16), (3, 4, 6, 16), (2, 2, 5, 32),
                                            (1, 1, 3, 64), (2, 8, 8, 8)])
def test_adjoint_y_map(nz, nux, nuy, nuz):
    if not (nux % (64 // nuz) == 0):
        pytest.skip("the kernel keeps the consecutive map")
    kk = adjoint_y_map(nz, nux, nuy, nuz)
    assert np.array_equal(np.sort(kk), np.arange(len(kk)))          # a permutation
    jy = ((kk % (nux * nuy * nuz)) // nuz) % nuy
    w = jy.reshape(-1, 64)
    assert np.all(w == w[:, :1])                                     # one u_y per wave

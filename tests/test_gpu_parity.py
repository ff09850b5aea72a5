"""Parity of the HIP path (through the C ABI) with the CPU FP64 oracle.

Floating-point bars:
  * SpMM: elementwise |W_gpu - W_ref| <= gamma_{z_i + 2} (|H| |V|)_i, the
    standard forward-error bound of a length-z_i dot product (u = 2^-53 for
    float64, 2^-24 for float32 accumulation), with W_ref the exact product of
    the same (rounded) inputs computed by the oracle;
  * tall-skinny products and the band eigensolver: FP64 results within a small
    multiple of n * u of numpy;
  * eigenvalues: 1e-10 relative on the float64 path, 1e-5 relative on the
    float32 path (against the oracle on the float32-rounded matrix);
  * residuals ||H x - theta x|| <= tol * ||H||_est, recomputed on the host.
"""
import numpy as np
import pytest

import synthgen
import oracle

pytestmark = pytest.mark.gpu

U64 = 2.0 ** -53
U32 = 2.0 ** -24
# blocks after the last block of a convergence check at which the solve reads
# it, for problems of fewer than 2^19 rows (the tests' sizes)
CHECK_LAG = 4


def note(msg):
    print("[case] " + msg, flush=True)


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available()
    return t


@pytest.fixture(scope="module")
def bbl(torch):
    import paper_2210_15763_amd as m
    m.load_library()
    return m


def gamma(m, u):
    return m * u / (1 - m * u)


def dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


# ------------------------------------------------------------------- SpMM
@pytest.mark.parametrize("nvec", [1, 3, 4, 8, 10, 12, 16, 32])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_spmm_matches_oracle_within_dot_product_bound(torch, bbl, nvec, prec):
    note("spmm n=20000 z~40 nvec=%d %s" % (nvec, prec))
    H = synthgen.generate(20000, 400, 20, 0.7, 11)
    V = synthgen.gaussian_block(H.n, nvec, 5)
    if prec == "f32":
        V = V.astype(np.float32).astype(np.float64)
        Href = H.as_float32_values()
        Hd = bbl.DeviceCSR.from_host(H, "float32")
        Vd = dev(torch, V.astype(np.float32))
        u = U32
    else:
        Href = H
        Hd = bbl.DeviceCSR.from_host(H, "float64")
        Vd = dev(torch, V)
        u = U64
    W = bbl.spmm(Hd, Vd).double().cpu().numpy()
    ref = oracle.spmm(Href, V)
    scale = oracle.spmm_abs(Href, V)
    z = np.diff(H.row_ptr)[:, None]
    bound = gamma(z + 2, u) * scale + 1e-300
    assert np.all(np.abs(W - ref) <= bound), np.max(np.abs(W - ref) / bound)


@pytest.mark.parametrize("nvec,block_rows,prec,q,p", [
    (8, 400, "f32", 20, 0.7), (8, 400, "f64", 20, 0.7), (1, 400, "f32", 20, 0.7),
    (4, 333, "f32", 20, 0.7), (10, 400, "f32", 20, 0.7), (16, 400, "f32", 20, 0.7),
    (2, 400, "f64", 20, 0.7), (16, 400, "f64", 20, 0.7), (8, 3000, "f32", 20, 0.7),
    (1, 25000, "f32", 20, 0.7),
    # long rows (~285 entries: several steps of staged entries per row) and
    # rows with most entries outside the staged blocks (several remote steps)
    (8, 400, "f32", 150, 0.7), (8, 400, "f32", 150, 0.1), (4, 400, "f32", 150, 0.3),
    (8, 1000, "f32", 105, 0.7), (10, 1000, "f32", 105, 0.7),
    (16, 1000, "f32", 105, 0.7), (16, 333, "f32", 150, 0.3), (12, 1000, "f32", 105, 0.7),
    (12, 400, "f32", 150, 0.3),
    # float64 plans through the pipelined passes (rows of 4 and 8 doubles)
    (4, 400, "f64", 20, 0.7), (4, 400, "f64", 150, 0.3), (8, 1000, "f64", 105, 0.7),
    (8, 333, "f64", 150, 0.3)])
def test_planned_spmm_matches_oracle(torch, bbl, nvec, block_rows, prec, q, p):
    """Rows reordered per group, partner blocks staged in LDS: the same sums
    in another order, so the dot-product bound holds entry by entry (groups
    of 333 rows straddle the generator's 400-row sectors; 3000-row groups
    leave a ragged last group; 25000 rows make one group larger than n)."""
    note("planned spmm block_rows=%d nvec=%d %s q=%d p=%.1f" % (block_rows, nvec, prec, q, p))
    H = synthgen.generate(20000, 400 if block_rows != 1000 else 1000, q, p, 11)
    dt = "float32" if prec == "f32" else "float64"
    Hd = bbl.DeviceCSR.from_host(H, dt, block_rows=block_rows)
    plan = bbl.spmm_plan(Hd, nvec)
    per_block = block_rows * nvec * (4 if prec == "f32" else 8)
    expect = min(5, 160 * 1024 // per_block)
    if nvec == 16 and prec == "f32":
        s16 = min(5, (160 * 1024 // 64 - 1) // block_rows)
        if 1 <= s16 < 3:
            # two 16-wide blocks per set fit beside the zero row: a multi-set
            # plan, one pass with lane pairs
            expect = s16
            assert plan.c.nsets > 0
        else:
            # two 8-column passes: a slot holds 8 columns, beside the zero row
            s8 = min(5, (160 * 1024 // 32 - 1) // block_rows)
            if s8 >= 1 and s8 * block_rows <= 65536:
                expect = s8
    assert plan.slots == expect
    V = synthgen.gaussian_block(H.n, nvec, 5)
    Vd = dev(torch, V.astype(np.float32) if prec == "f32" else V)
    W = bbl.spmm_planned(plan, Vd).double().cpu().numpy()
    W2 = bbl.spmm_planned(plan, Vd).double().cpu().numpy()
    assert np.array_equal(W, W2)
    Href = H.as_float32_values() if prec == "f32" else H
    Vr = V.astype(np.float32).astype(np.float64) if prec == "f32" else V
    u = U32 if prec == "f32" else U64
    z = np.diff(H.row_ptr)[:, None]
    bound = gamma(z + 2, u) * oracle.spmm_abs(Href, Vr) + 1e-300
    assert np.all(np.abs(W - oracle.spmm(Href, Vr)) <= bound)


@pytest.mark.parametrize("n,R,q,p,nvec,block_rows", [
    (40000, 2000, 105, 0.7, 8, 2000), (40000, 2000, 105, 0.7, 16, 2000),
    (40000, 2000, 105, 0.7, 10, 2000), (40000, 1000, 60, 0.5, 4, 5000),
    # many small sectors: groups reach more column blocks than the sets
    # hold, so many entries take the gather pass
    (60000, 200, 40, 0.3, 8, 2000), (60000, 200, 40, 0.3, 16, 2000),
    # a ragged last group
    (41000, 1000, 60, 0.7, 8, 3000),
    # short rows (~50 entries, half of them far from the row's sector)
    (60000, 2000, 25, 0.5, 8, 2000), (44000, 2000, 25, 0.5, 10, 2000),
    (44000, 2000, 25, 0.5, 16, 2000)])
def test_multiset_planned_spmm_matches_oracle(torch, bbl, n, R, q, p, nvec, block_rows):
    """The multi-set plan (fewer than three column blocks fit in LDS per set):
    nsets sets of the group's busiest blocks staged one after the other, the
    rest gathered; the same sums in another order, so the dot-product bound
    holds entry by entry; bitwise reproducible."""
    note("multi-set planned spmm n=%d block_rows=%d nvec=%d p=%.1f" % (n, block_rows, nvec, p))
    H = synthgen.generate(n, R, q, p, 13)
    Hd = bbl.DeviceCSR.from_host(H, "float32", block_rows=block_rows)
    plan = bbl.spmm_plan(Hd, nvec)
    # 16 vectors: sets of 16-wide rows (lane pairs) when one block fits
    # beside the zero row, else 8-column halves
    bk = 8 if nvec == 16 and (block_rows + 1) * 64 > 160 * 1024 else nvec
    s = min(5, (160 * 1024 // (bk * 4) - 1) // block_rows)
    assert plan.c.nsets > 0 and plan.slots == s
    assert plan.c.nsets == min(16 // s, -(-10 // s))
    V = synthgen.gaussian_block(H.n, nvec, 5)
    Vd = dev(torch, V.astype(np.float32))
    W = bbl.spmm_planned(plan, Vd).double().cpu().numpy()
    W2 = bbl.spmm_planned(plan, Vd).double().cpu().numpy()
    assert np.array_equal(W, W2)
    Href = H.as_float32_values()
    Vr = V.astype(np.float32).astype(np.float64)
    z = np.diff(H.row_ptr)[:, None]
    bound = gamma(z + 2, U32) * oracle.spmm_abs(Href, Vr) + 1e-300
    assert np.all(np.abs(W - oracle.spmm(Href, Vr)) <= bound)


def test_multiset_planned_solve(torch, bbl):
    """A b = 16 FP32 solve with thick restart through the multi-set plan
    (2000-row sectors, the n = 2e7 shape in small): host FP64 residuals and
    the same eigenvalues as through the plain CSR kernel."""
    note("multi-set planned solve b=16")
    H = synthgen.generate(60000, 2000, 105, 0.7, 4)
    Hp = bbl.DeviceCSR.from_host(H, "float32", block_rows=2000)
    plan = bbl.spmm_plan(Hp, 16)
    assert plan.c.nsets > 0
    P = bbl.random_pivot(H.n, 16, synthgen.pivot_key(3))
    rp = bbl.block_lanczos(Hp, P, 10, 1e-6, m_max=20, restart_keep=32, spmm_plan=plan)
    r = bbl.block_lanczos(Hp, P, 10, 1e-6, m_max=20, restart_keep=32)
    assert rp.converged and r.converged, (rp.stats, r.stats)
    hn = rp.stats["hnorm_est"]
    np.testing.assert_allclose(rp.eigvals, r.eigvals, rtol=0, atol=2e-6 * hn)
    res = oracle.ritz_residuals(H.as_float32_values(), rp.eigvecs.cpu().numpy(), rp.eigvals)
    assert np.all(res <= 1e-6 * hn), res / hn


def test_spmm_plan_layout_and_errors(torch, bbl):
    note("spmm plan layout")
    H = synthgen.generate(12000, 400, 20, 0.7, 3)
    Hd = bbl.DeviceCSR.from_host(H, "float32", block_rows=400)
    plan = bbl.spmm_plan(Hd, 8)
    # n_local sits in the plan buffer right after the block table
    off = plan.c.n_local - plan.mem.data_ptr()
    assert off == ((plan.mem.data_ptr() + 255) // 256 * 256 - plan.mem.data_ptr()
                   + -(-(30 * 2 * plan.slots * 4) // 256) * 256)
    nl = plan.mem[off:off + 4 * H.n].view(torch.int32).cpu().numpy()
    lens = np.diff(H.row_ptr)
    assert np.all(nl >= 0) and np.all(nl <= lens)
    # own sector (70 % of draws) plus the three busiest partners
    assert nl.sum() / lens.sum() > 0.75
    # the 16-bit copy of the LDS row indices matches the 32-bit one on every
    # staged entry (the first n_local entries of each row)
    assert plan.c.local16 == 1
    oc = plan.c.col - plan.mem.data_ptr()
    ol = plan.c.lcol - plan.mem.data_ptr()
    col2 = plan.mem[oc:oc + 4 * H.nnz].view(torch.int32).cpu().numpy()
    lcol = plan.mem[ol:ol + 2 * H.nnz].view(torch.int16).cpu().numpy().view(np.uint16)
    rows = np.repeat(np.arange(H.n), lens)
    staged = np.arange(H.nnz) - np.asarray(H.row_ptr)[rows] < nl[rows]
    assert staged.sum() == nl.sum()
    assert np.array_equal(lcol[staged].astype(np.int64), col2[staged].astype(np.int64))
    assert np.all(col2[staged] < plan.slots * 400)
    # block table: per group its own block, then the other blocks by entry
    # count (set A: the first `slots`, set B: the next `slots`)
    ob = plan.c.blocks - plan.mem.data_ptr()
    S = plan.slots
    blk = plan.mem[ob:ob + 4 * 30 * 2 * S].view(torch.int32).cpu().numpy().reshape(30, 2 * S)
    cb = np.asarray(H.col) // 400
    for g in (0, 7, 29):
        m = rows // 400 == g
        cnt = np.bincount(cb[m], minlength=30)
        assert blk[g, 0] == g
        others = blk[g, 1:][blk[g, 1:] >= 0]
        assert len(set(others.tolist())) == len(others) and g not in others
        c = cnt[others]
        assert np.all(np.diff(c) <= 0) and np.all(c > 0)
        rest = np.setdiff1d(np.nonzero(cnt)[0], np.concatenate([[g], others]))
        assert len(rest) == 0 or cnt[rest].max() <= c.min()
    # per-row descriptors: first entry, first set-B entry, first remaining
    # entry, end, relative to the row group's first entry rounded down to 8
    od = plan.c.rdesc - plan.mem.data_ptr()
    d = plan.mem[od:od + 16 * H.n].view(torch.int32).cpu().numpy().reshape(-1, 4).astype(np.int64)
    rp = np.asarray(H.row_ptr)
    gb = rp[(np.arange(H.n) // 400) * 400] & ~7
    assert np.array_equal(d[:, 0], rp[:-1] - gb)
    assert np.array_equal(d[:, 1], rp[:-1] + nl - gb)
    assert np.array_equal(d[:, 3], rp[1:] - gb)
    assert np.all(d[:, 1] <= d[:, 2]) and np.all(d[:, 2] <= d[:, 3])
    # set-B entries: global columns in col, in-set LDS rows in lcol, in order;
    # the rest: global columns outside both sets
    pos = np.arange(H.nnz) - gb[rows]
    inb = (pos >= d[rows, 1]) & (pos < d[rows, 2])
    rem = pos >= d[rows, 2]
    setb = blk[rows // 400, S:]
    gcol = col2.astype(np.int64)
    okb = (gcol[inb][:, None] // 400 == setb[inb]).any(axis=1)
    assert okb.all()
    k = np.argmax(gcol[inb][:, None] // 400 == setb[inb], axis=1)
    assert np.array_equal(lcol[inb].astype(np.int64), k * 400 + gcol[inb] % 400)
    allb = blk[rows // 400]
    assert not (gcol[rem][:, None] // 400 == allb[rem]).any()
    # the dense copy of the set-B entries: each group's rows in order, no gaps
    G = 400
    ogr = plan.c.bgroup - plan.mem.data_ptr()
    bg = plan.mem[ogr:ogr + 8 * 31].view(torch.int64).cpu().numpy()
    obr = plan.c.brow - plan.mem.data_ptr()
    br = plan.mem[obr:obr + 8 * H.n].view(torch.int32).cpu().numpy().reshape(-1, 2).astype(np.int64)
    nbr = d[:, 2] - d[:, 1]
    assert bg[0] == 0 and np.array_equal(np.diff(bg), np.add.reduceat(nbr, np.arange(0, H.n, G)))
    first = (bg[np.arange(H.n) // G] & ~7) + br[:, 0]
    assert np.array_equal(br[:, 1] - br[:, 0], nbr)
    assert np.array_equal(first[1:][nbr[:-1] >= 0], (first + nbr)[:-1])
    obl = plan.c.blcol - plan.mem.data_ptr()
    obv = plan.c.bval - plan.mem.data_ptr()
    nb_all = int(bg[-1])
    bl = plan.mem[obl:obl + 2 * nb_all].view(torch.int16).cpu().numpy().view(np.uint16)
    ov = plan.c.val - plan.mem.data_ptr()
    val2 = plan.mem[ov:ov + 4 * H.nnz].view(torch.float32).cpu().numpy()
    bv = plan.mem[obv:obv + 4 * nb_all].view(torch.float32).cpu().numpy()
    assert np.array_equal(bl, lcol[inb]) and np.array_equal(bv, val2[inb])
    # the dense copy of the set-A entries, likewise
    oag = plan.c.agroup - plan.mem.data_ptr()
    ag = plan.mem[oag:oag + 8 * 31].view(torch.int64).cpu().numpy()
    oar = plan.c.arow - plan.mem.data_ptr()
    ar = plan.mem[oar:oar + 8 * H.n].view(torch.int32).cpu().numpy().reshape(-1, 2).astype(np.int64)
    assert ag[0] == 0 and np.array_equal(np.diff(ag), np.add.reduceat(nl.astype(np.int64), np.arange(0, H.n, G)))
    assert np.array_equal(ar[:, 1] - ar[:, 0], nl)
    afirst = (ag[np.arange(H.n) // G] & ~7) + ar[:, 0]
    assert np.array_equal(afirst[1:], (afirst + nl)[:-1])
    na_all = int(ag[-1])
    oal = plan.c.alcol - plan.mem.data_ptr()
    oav = plan.c.aval - plan.mem.data_ptr()
    al = plan.mem[oal:oal + 2 * na_all].view(torch.int16).cpu().numpy().view(np.uint16)
    av = plan.mem[oav:oav + 4 * na_all].view(torch.float32).cpu().numpy()
    assert np.array_equal(al, lcol[staged]) and np.array_equal(av, val2[staged])
    # the list of rows with entries outside both sets: {row, count, first}
    org = plan.c.rgroup - plan.mem.data_ptr()
    rg = plan.mem[org:org + 8 * 31].view(torch.int64).cpu().numpy()
    has = d[:, 3] > d[:, 2]
    assert rg[0] == 0 and np.array_equal(np.diff(rg), np.add.reduceat(has.astype(np.int64), np.arange(0, H.n, G)))
    orl = plan.c.rlist - plan.mem.data_ptr()
    rl = plan.mem[orl:orl + 16 * int(rg[-1])].view(torch.int32).cpu().numpy().reshape(-1, 4)
    want = np.nonzero(has)[0]
    assert np.array_equal(rl[:, 0], want)
    assert np.array_equal(rl[:, 1], (d[want, 3] - d[want, 2]))
    firsts = (rl[:, 2].astype(np.int64) & 0xffffffff) | (rl[:, 3].astype(np.int64) << 32)
    assert np.array_equal(firsts, gb[want] + d[want, 2])
    # the (row, column) pairs outside set A are those of H
    ocol = np.asarray(H.col).astype(np.int64)
    nota = ~(ocol[:, None] // 400 == blk[rows // 400, :S]).any(axis=1)
    assert np.array_equal(np.sort(rows[nota] * H.n + ocol[nota]),
                          np.sort(rows[inb | rem] * H.n + gcol[inb | rem]))
    with pytest.raises(bbl.BblError):
        bbl.spmm_plan(bbl.DeviceCSR.from_host(H, "float32"), 8)          # no hint
    with pytest.raises(bbl.BblError):
        bbl.spmm_plan(Hd, 3)                                             # no kernel width 3


def test_planned_spmm_ignores_rows_of_v_it_does_not_use(torch, bbl):
    """Lanes without an entry of their own must not pick up values of V: with
    an infinite row of V, exactly the rows of H that reference it are not
    finite, and every other row keeps its dot-product bound."""
    note("planned spmm with an infinite row of V")
    H = synthgen.generate(20000, 400, 60, 0.7, 12)
    Hd = bbl.DeviceCSR.from_host(H, "float32", block_rows=400)
    plan = bbl.spmm_plan(Hd, 8)
    V = synthgen.gaussian_block(H.n, 8, 6).astype(np.float32)
    bad = [0, 401, 19999]
    V[bad] = np.inf
    W = bbl.spmm_planned(plan, dev(torch, V)).double().cpu().numpy()
    rows = np.repeat(np.arange(H.n), np.diff(H.row_ptr))
    touched = np.zeros(H.n, bool)
    touched[rows[np.isin(np.asarray(H.col), bad)]] = True
    assert touched.sum() > 0 and (~touched).sum() > 0
    assert not np.any(np.isfinite(W[touched]).all(axis=1))
    ok = ~touched
    assert np.all(np.isfinite(W[ok]))
    Vr = V.astype(np.float64)
    Vr[bad] = 0.0
    Href = H.as_float32_values()
    z = np.diff(H.row_ptr)[:, None]
    bound = gamma(z + 2, U32) * oracle.spmm_abs(Href, Vr) + 1e-300
    assert np.all((np.abs(W - oracle.spmm(Href, Vr)) <= bound)[ok])


def test_spmm_ragged_rows_and_empty_rows(torch, bbl):
    note("spmm ragged/empty rows")
    rng = np.random.default_rng(0)
    n = 3001
    lens = rng.integers(0, 300, n)
    lens[::17] = 0
    lens[5] = 1000
    rp = np.zeros(n + 1, np.int64)
    rp[1:] = np.cumsum(lens)
    col = np.concatenate([np.sort(rng.choice(n, size=l, replace=False)) for l in lens]).astype(np.int32)
    val = rng.standard_normal(rp[-1])
    H = synthgen.CSR(n, rp, col, val)
    V = rng.standard_normal((n, 8))
    W = bbl.spmm(bbl.DeviceCSR.from_host(H, "float64"), dev(torch, V)).cpu().numpy()
    ref = oracle.spmm(H, V)
    bound = gamma(lens[:, None] + 2, U64) * oracle.spmm_abs(H, V) + 1e-300
    assert np.all(np.abs(W - ref) <= bound)
    assert np.all(W[lens == 0] == 0.0)


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_spmm_unaligned_arrays(torch, bbl, prec):
    """Column and value arrays that do not start on a 16-byte boundary (views
    one element into a larger buffer): the plain kernel loads them per entry."""
    note("spmm unaligned col/val %s" % prec)
    H = synthgen.generate(6000, 400, 20, 0.7, 13)
    dt = np.float32 if prec == "f32" else np.float64
    colb = torch.from_numpy(np.concatenate([[0], H.col]).astype(np.int32)).cuda()
    valb = torch.from_numpy(np.concatenate([[0.0], H.val]).astype(dt)).cuda()
    Hd = bbl.DeviceCSR(H.n, torch.from_numpy(np.asarray(H.row_ptr, np.int64)).cuda(), colb[1:],
                       valb[1:])
    assert Hd.col.data_ptr() % 16 != 0
    V = synthgen.gaussian_block(H.n, 8, 2)
    Vd = dev(torch, V.astype(dt))
    W = bbl.spmm(Hd, Vd).double().cpu().numpy()
    Href = H.as_float32_values() if prec == "f32" else H
    Vr = V.astype(dt).astype(np.float64)
    u = U32 if prec == "f32" else U64
    bound = gamma(np.diff(H.row_ptr)[:, None] + 2, u) * oracle.spmm_abs(Href, Vr) + 1e-300
    assert np.all(np.abs(W - oracle.spmm(Href, Vr)) <= bound)


def test_spmm_bitwise_reproducible(torch, bbl):
    note("spmm reproducibility")
    H = synthgen.generate(40000, 1000, 50, 0.7, 3)
    Hd = bbl.DeviceCSR.from_host(H, "float32")
    V = dev(torch, synthgen.gaussian_block(H.n, 8, 1).astype(np.float32))
    a = bbl.spmm(Hd, V).cpu().numpy()
    b = bbl.spmm(Hd, V).cpu().numpy()
    assert np.array_equal(a, b)


# ------------------------------------------------------- tall-skinny products
@pytest.mark.parametrize("bx,nblk,ny,xf32", [(8, 3, 8, True), (16, 2, 16, True), (4, 5, 4, False),
                                             (10, 3, 10, True), (8, 1, 20, False),
                                             (8, 7, 8, False), (8, 9, 8, True), (8, 37, 8, True),
                                             (8, 1, 8, True), (8, 1, 8, False), (4, 1, 4, True),
                                             (8, 23, 10, True), (8, 4, 10, False),
                                             (4, 20, 4, False), (16, 1, 16, True),
                                             (16, 1, 16, False), (16, 3, 16, False),
                                             (16, 5, 16, True), (16, 40, 16, True),
                                             (10, 1, 10, True), (10, 1, 10, False),
                                             (10, 20, 10, True)])
def test_gram_and_update_match_numpy(torch, bbl, bx, nblk, ny, xf32):
    """(5003 rows with 16 or more blocks take the wave-split update.)"""
    note("gram/update bx=%d nblk=%d ny=%d f32=%s" % (bx, nblk, ny, xf32))
    rng = np.random.default_rng(bx * 100 + nblk)
    n = 5003  # several tiles plus a ragged tail
    Xb = rng.standard_normal((nblk, n, bx))
    if xf32:
        Xb = Xb.astype(np.float32).astype(np.float64)
    Y = rng.standard_normal((n, ny))
    Xd = dev(torch, Xb.astype(np.float32) if xf32 else Xb)
    Yd = dev(torch, Y)
    Xwide = np.concatenate(list(Xb), axis=1)  # n x (nblk*bx)
    C = bbl.gram(Xd, nblk, bx, Yd).cpu().numpy()
    Cref = Xwide.T @ Y
    assert np.max(np.abs(C - Cref)) <= 64 * n * U64 * np.max(np.abs(Xwide).T @ np.abs(Y))
    Cm = rng.standard_normal((nblk * bx, ny))
    Out = torch.empty_like(Yd)
    bbl.block_update(Xd, nblk, bx, dev(torch, Cm), -1.0, Yd, 1.0, Out)
    ref = Y - Xwide @ Cm
    tol = 64 * nblk * bx * U64 * (np.abs(Y) + np.abs(Xwide) @ np.abs(Cm))
    assert np.all(np.abs(Out.cpu().numpy() - ref) <= tol)
    # beta = 0 and float32 output
    Out32 = torch.empty((n, ny), dtype=torch.float32, device="cuda")
    bbl.block_update(Xd, nblk, bx, dev(torch, Cm), 1.0, None, 0.0, Out32)
    np.testing.assert_allclose(Out32.double().cpu().numpy(), Xwide @ Cm, rtol=2e-6, atol=2e-6 * np.abs(Xwide @ Cm).max())


@pytest.mark.parametrize("bx", [8, 10])
def test_gram_at_a_row_count_past_the_short_row_path(torch, bbl, bx):
    """The 8- and 10-wide matrix-core grams at 700,003 rows (row chunks of 256
    rows and more, two row groups in flight; the parity case above, at 5003
    rows, takes the short-row launch) against numpy in float64."""
    note("gram bx=%d n=700003" % bx)
    rng = np.random.default_rng(bx)
    n, nblk = 700_003, 5
    Xb = rng.standard_normal((nblk, n, bx)).astype(np.float32)
    Y = rng.standard_normal((n, bx))
    C = bbl.gram(dev(torch, Xb), nblk, bx, dev(torch, Y)).cpu().numpy()
    Xwide = np.concatenate([Xb[i].astype(np.float64) for i in range(nblk)], axis=1)
    Cref = Xwide.T @ Y
    bound = 64 * n * U64 * (np.abs(Xwide).T @ np.abs(Y))
    assert np.all(np.abs(C.reshape(Cref.shape) - Cref) <= bound)


@pytest.mark.parametrize("n", [1, 7, 17, 33])
def test_sixteen_wide_products_on_tiny_row_counts(torch, bbl, n):
    """The 16-wide matrix-core gram and update on fewer rows than one 16-row
    tile (and a tile and a bit): masked rows contribute nothing; the update
    also in place (Yin is Yout), as the recurrence calls it."""
    note("16-wide gram/update n=%d" % n)
    rng = np.random.default_rng(500 + n)
    nblk = 3
    Xb = rng.standard_normal((nblk, n, 16)).astype(np.float32)
    Y = rng.standard_normal((n, 16))
    Xd, Yd = dev(torch, Xb), dev(torch, Y)
    Xwide = np.concatenate(list(Xb.astype(np.float64)), axis=1)
    C = bbl.gram(Xd, nblk, 16, Yd).cpu().numpy()
    np.testing.assert_allclose(C, Xwide.T @ Y, rtol=0, atol=64 * n * U64 * np.abs(Xwide).T.dot(np.abs(Y)).max() + 1e-300)
    Cm = rng.standard_normal((nblk * 16, 16))
    bbl.block_update(Xd, nblk, 16, dev(torch, Cm), -1.0, Yd, 1.0, Yd)
    ref = Y - Xwide @ Cm
    tol = 64 * nblk * 16 * U64 * (np.abs(Y) + np.abs(Xwide) @ np.abs(Cm))
    assert np.all(np.abs(Yd.cpu().numpy() - ref) <= tol)


@pytest.mark.parametrize("bx,nblk", [(16, 1), (16, 2), (8, 1)])
def test_gram_of_float32_operands_matches_numpy(torch, bbl, bx, nblk):
    """The recurrence's A_J = V_J^T W takes both operands in float32 (the
    SpMM's output); 16-wide blocks run it on FP64 matrix cores."""
    note("gram f32 x f32 bx=%d nblk=%d" % (bx, nblk))
    rng = np.random.default_rng(77 + bx + nblk)
    n = 4099
    Xb = rng.standard_normal((nblk, n, bx)).astype(np.float32)
    Y = rng.standard_normal((n, bx)).astype(np.float32)
    C = bbl.gram(dev(torch, Xb), nblk, bx, dev(torch, Y)).cpu().numpy()
    Xwide = np.concatenate(list(Xb.astype(np.float64)), axis=1)
    Cref = Xwide.T @ Y.astype(np.float64)
    assert np.max(np.abs(C - Cref)) <= 64 * n * U64 * np.max(np.abs(Xwide).T @ np.abs(Y))


# ---------------------------------------------------------- band eigensolver
def band_from_dense(T, kd):
    N = T.shape[0]
    band = np.zeros((N, kd + 1))
    for d in range(kd + 1):
        band[d:, d] = np.diagonal(T, -d)
    return band


@pytest.mark.parametrize("N,kd,k", [(200, 4, 10), (640, 8, 10), (333, 16, 12), (40, 8, 32),
                                    (17, 4, 17)])
def test_band_eig_matches_dense_eigh(torch, bbl, N, kd, k):
    note("band eig N=%d kd=%d k=%d" % (N, kd, k))
    rng = np.random.default_rng(N + kd)
    T = np.zeros((N, N))
    for d in range(kd + 1):
        v = rng.standard_normal(N - d) * (3.0 if d == 0 else 1.0)
        T += np.diag(v, -d) + (np.diag(v, d) if d else 0)
    T += np.diag(np.linspace(-20, 20, N))
    lam, S = np.linalg.eigh(T)
    theta, Sg, top = bbl.band_eig(dev(torch, band_from_dense(T, kd)), N, kd, k)
    nrm = max(abs(lam[0]), abs(lam[-1]))
    np.testing.assert_allclose(theta, lam[:k], rtol=0, atol=1e-12 * nrm)
    assert abs(top - lam[-1]) <= 1e-12 * nrm
    Sg = Sg.cpu().numpy()
    assert np.max(np.linalg.norm(T @ Sg - Sg * theta, axis=0)) <= 1e-11 * nrm
    assert np.max(np.abs(Sg.T @ Sg - np.eye(k))) <= 1e-12


@pytest.mark.parametrize("kd", [4, 6])
def test_band_eig_double_eigenvalues(torch, bbl, kd):
    """T = diag(B, B): every eigenvalue twice.  Inverse iteration at equal
    shifts must still give an orthonormal basis of each 2-d eigenspace."""
    note("band eig with doubled spectrum kd=%d" % kd)
    rng = np.random.default_rng(11 + kd)
    m = 150
    B = np.zeros((m, m))
    for d in range(kd + 1):
        v = rng.standard_normal(m - d)
        B += np.diag(v, -d) + (np.diag(v, d) if d else 0)
    T = np.zeros((2 * m, 2 * m))
    T[:m, :m] = B
    T[m:, m:] = B
    lam = np.linalg.eigvalsh(T)
    theta, Sg, top = bbl.band_eig(dev(torch, band_from_dense(T, kd)), 2 * m, kd, 10)
    nrm = max(abs(lam[0]), abs(lam[-1]))
    np.testing.assert_allclose(theta, lam[:10], rtol=0, atol=1e-12 * nrm)
    Sg = Sg.cpu().numpy()
    assert np.max(np.abs(Sg.T @ Sg - np.eye(10))) <= 1e-12
    assert np.max(np.linalg.norm(T @ Sg - Sg * theta, axis=0)) <= 1e-11 * nrm


def test_band_eig_on_lanczos_band_matrix(torch, bbl):
    note("band eig on an oracle block-Lanczos band matrix")
    H = synthgen.generate(20000, 400, 20, 0.7, 0)
    P = synthgen.gaussian_block(H.n, 4, 3)
    res = oracle.block_lanczos(H, P, 4, 1e-300, 60, keep=True)
    from oracle.lanczos import band_matrix
    T = band_matrix(res.A, res.B[:len(res.A) - 1])
    lam = np.linalg.eigvalsh(T)
    theta, Sg, top = bbl.band_eig(dev(torch, band_from_dense(T, 7)), T.shape[0], 7, 10)
    np.testing.assert_allclose(theta, lam[:10], rtol=0, atol=1e-12 * abs(lam[0]))


# ---------------------------------------------------------------- pivots
def test_random_pivot_matches_generator_stream(torch, bbl):
    note("random pivot")
    key = synthgen.pivot_key(7)
    g = bbl.random_pivot(100003, 8, key).cpu().numpy()
    ref = synthgen.gaussian_block(100003, 8, key)
    assert np.max(np.abs(g - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_bootstrap_pivot_spans_truncated_eigenvectors(torch, bbl):
    note("bootstrap pivot n=20000 n_t=2000 b=4")
    H = synthgen.WORKLOADS["small_fp64_n2e4"].generate()
    Hd = bbl.DeviceCSR.from_host(H, "float64")
    P, st = bbl.bootstrap_pivot(Hd, 2000, 4, 1e-10, m_max=400)
    P = P.cpu().numpy()
    assert np.all(P[2000:] == 0)
    Pref = oracle.bootstrap_pivot(H, 2000, 4)
    sv = np.linalg.svd(Pref.T @ P, compute_uv=False)
    assert sv.min() > 1 - 1e-9, sv
    assert st["converged"] == 1


# ----------------------------------------------------------- block Lanczos
def test_small_fp64_workload_matches_oracle(torch, bbl):
    """n = 2e4, ~40 nnz/row, FP64 throughout, b = k = 4, tol 1e-8, bootstrap
    pivot from the leading 2000 x 2000 block."""
    w = synthgen.WORKLOADS["small_fp64_n2e4"]
    note("small FP64 workload end to end")
    H = w.generate()
    Hd = bbl.DeviceCSR.from_host(H, "float64")
    P, _ = bbl.bootstrap_pivot(Hd, w.n_trunc, w.nvec, w.tol, m_max=w.m_max)
    r = bbl.block_lanczos(Hd, P, w.k, w.tol, m_max=w.m_max)
    assert r.converged, r.stats
    Pref = oracle.bootstrap_pivot(H, w.n_trunc, w.nvec)
    ro = oracle.block_lanczos(H, Pref, w.k, w.tol, w.m_max)
    assert ro.converged
    np.testing.assert_allclose(r.eigvals, ro.eigvals, rtol=1e-10)
    X = r.eigvecs.cpu().numpy()
    res_host = oracle.ritz_residuals(H, X, r.eigvals)
    assert np.all(res_host <= w.tol * r.stats["hnorm_est"])
    np.testing.assert_allclose(r.residuals, res_host, rtol=1e-6, atol=1e-3 * w.tol * r.stats["hnorm_est"])
    sv = np.linalg.svd(ro.eigvecs.T @ X, compute_uv=False)
    assert sv.min() > 1 - 1e-8
    # same pivot as the oracle: iteration counts agree to one block
    r2 = bbl.block_lanczos(Hd, dev(torch, Pref), w.k, w.tol, m_max=w.m_max, check_every=1)
    assert abs(r2.stats["iters"] - ro.iters) <= 1, (r2.stats["iters"], ro.iters)
    np.testing.assert_allclose(r2.eigvals, ro.eigvals, rtol=1e-10)


def test_spmm_timing_flag_times_every_block_and_changes_nothing(torch, bbl):
    note("BBL_FLAG_TIME_SPMM")
    w = synthgen.WORKLOADS["small_fp64_n2e4"]
    H = w.generate()
    Hd = bbl.DeviceCSR.from_host(H, "float64")
    P = bbl.random_pivot(H.n, 4, synthgen.pivot_key(3))
    a = bbl.block_lanczos(Hd, P, 4, 1e-8, m_max=300)
    t = bbl.block_lanczos(Hd, P, 4, 1e-8, m_max=300, time_spmm=True)
    assert a.stats["spmm_timed"] == 0 and a.stats["spmm_ms"] == 0.0
    # every block built is timed: the returned pairs' blocks, plus at most the
    # CHECK_LAG built while the deciding check ran and its last block was
    # verified
    assert t.stats["iters"] <= t.stats["spmm_timed"] <= t.stats["iters"] + CHECK_LAG
    assert t.stats["spmm_ms"] > 0
    assert np.array_equal(a.eigvals, t.eigvals) and a.stats["iters"] == t.stats["iters"]


def test_random_pivot_finds_same_eigenvalues(torch, bbl):
    note("random vs bootstrap pivot agree on the eigenvalue set")
    w = synthgen.WORKLOADS["small_fp64_n2e4"]
    H = w.generate()
    Hd = bbl.DeviceCSR.from_host(H, "float64")
    Pr = bbl.random_pivot(H.n, 4, synthgen.pivot_key(0))
    r = bbl.block_lanczos(Hd, Pr, 4, 1e-8, m_max=300)
    Pref = synthgen.gaussian_block(H.n, 4, synthgen.pivot_key(0))
    ro = oracle.block_lanczos(H, Pref, 4, 1e-8, 300)
    assert r.converged and ro.converged
    np.testing.assert_allclose(r.eigvals, ro.eigvals, rtol=1e-10)


def test_fp32_path_matches_oracle_on_rounded_matrix(torch, bbl):
    note("FP32 path n=40000 z~200 b=8 k=10")
    H = synthgen.generate(40000, 1000, 105, 0.7, 2)
    Hd = bbl.DeviceCSR.from_host(H, "float32")
    P, _ = bbl.bootstrap_pivot(Hd, 4000, 8, 1e-6, m_max=200)
    r = bbl.block_lanczos(Hd, P, 10, 1e-6, m_max=200)
    assert r.converged, r.stats
    H32 = H.as_float32_values()
    Pref = oracle.bootstrap_pivot(H32, 4000, 8)
    ro = oracle.block_lanczos(H32, Pref, 10, 1e-6, 200)
    np.testing.assert_allclose(r.eigvals, ro.eigvals, rtol=1e-5)
    X = r.eigvecs.cpu().numpy()
    res_host = oracle.ritz_residuals(H32, X, r.eigvals)
    assert np.all(res_host <= 1e-6 * r.stats["hnorm_est"])
    # FP64 run of the same matrix
    Hd64 = bbl.DeviceCSR.from_host(H32, "float64")
    r64 = bbl.block_lanczos(Hd64, P, 10, 1e-6, m_max=200)
    np.testing.assert_allclose(r.eigvals, r64.eigvals, rtol=1e-5)
    # the recurrence through the planned SpMM (sectors of 1000 rows)
    Hp = bbl.DeviceCSR.from_host(H, "float32", block_rows=1000)
    plan = bbl.spmm_plan(Hp, 8)
    rp = bbl.block_lanczos(Hp, P, 10, 1e-6, m_max=200, spmm_plan=plan)
    assert rp.converged
    np.testing.assert_allclose(rp.eigvals, ro.eigvals, rtol=1e-5)
    res_p = oracle.ritz_residuals(H32, rp.eigvecs.cpu().numpy(), rp.eigvals)
    assert np.all(res_p <= 1e-6 * rp.stats["hnorm_est"])
    with pytest.raises(bbl.BblError):       # a plan for another block width
        bbl.block_lanczos(Hp, P[:, :4].contiguous(), 4, 1e-6, m_max=50, spmm_plan=plan)


@pytest.mark.parametrize("block_rows", [1000, 400])
def test_planned_solve_at_sixteen_vectors(torch, bbl, block_rows):
    """b = 16 through the planned SpMM -- at 1000-row groups one pass over
    16-wide rows with lane pairs (a multi-set plan of two blocks per set), at
    400-row groups two passes over 8-column halves: residuals of the
    converged pairs recomputed on the host in FP64, and the same eigenvalues
    (within the residual bound) as the solve through the plain CSR kernel."""
    note("planned solve b=16 block_rows=%d" % block_rows)
    H = synthgen.generate(20000, 1000, 105, 0.7, 12)
    Hp = bbl.DeviceCSR.from_host(H, "float32", block_rows=block_rows)
    plan = bbl.spmm_plan(Hp, 16)
    if block_rows == 1000:
        assert plan.slots == 2 and plan.c.nsets > 0
    else:
        assert plan.slots == 5 and plan.c.nsets == 0
    P = bbl.random_pivot(H.n, 16, synthgen.pivot_key(3))
    rp = bbl.block_lanczos(Hp, P, 10, 1e-6, m_max=120, spmm_plan=plan)
    r = bbl.block_lanczos(Hp, P, 10, 1e-6, m_max=120)
    assert rp.converged and r.converged, (rp.stats, r.stats)
    hn = rp.stats["hnorm_est"]
    np.testing.assert_allclose(rp.eigvals, r.eigvals, rtol=0, atol=2e-6 * hn)
    res = oracle.ritz_residuals(H.as_float32_values(), rp.eigvecs.cpu().numpy(), rp.eigvals)
    assert np.all(res <= 1e-6 * hn), res / hn


def test_exact_eigenvector_pivot_deflates_and_converges_at_once(torch, bbl):
    note("exact-eigenvector pivot")
    H = synthgen.generate(1600, 400, 20, 0.7, 6)
    lam, X = np.linalg.eigh(H.to_dense())
    Hd = bbl.DeviceCSR.from_host(H, "float64")
    r = bbl.block_lanczos(Hd, dev(torch, X[:, :4]), 4, 1e-10, m_max=10, check_every=1)
    assert r.converged and r.stats["iters"] == 1
    assert r.stats["deflations"] == 4
    np.testing.assert_allclose(r.eigvals, lam[:4], rtol=1e-12)


def test_exhausted_invariant_subspace_takes_the_full_path(torch, bbl):
    """A pivot inside a 12-dimensional invariant subspace: the third block's
    W' is rounding noise inside the basis span, so that block needs the
    second Gram-Schmidt sweep and a full deflation -- the branches the fast
    path leaves to a redo on the full path."""
    note("exhausted invariant subspace n=412 b=4")
    A = synthgen.generate(12, 12, 4, 0.7, 5).to_dense() + 100.0 * np.eye(12)
    Bm = synthgen.generate(400, 100, 10, 0.7, 6).to_dense()
    D = np.zeros((412, 412))
    D[:12, :12] = A
    D[12:, 12:] = Bm
    rp = [0]
    cols, vals = [], []
    for i in range(412):
        nz = np.nonzero(D[i])[0]
        cols.append(nz)
        vals.append(D[i, nz])
        rp.append(rp[-1] + len(nz))
    H = synthgen.CSR(412, np.array(rp, np.int64), np.concatenate(cols).astype(np.int32),
                     np.concatenate(vals))
    P = np.zeros((412, 4))
    P[:12] = synthgen.gaussian_block(12, 4, 3)
    r = bbl.block_lanczos(bbl.DeviceCSR.from_host(H, "float64"), dev(torch, P), 4, 1e-10,
                          m_max=50)
    # the Krylov space of the pivot is the invariant subspace: its pairs are
    # exact (the coupling to the deflated block vanishes), as in the oracle
    ref = oracle.block_lanczos(H, P, 4, 1e-10, 50)
    assert ref.converged and ref.iters == 3 and ref.deflations == 4
    assert r.converged and r.stats["iters"] == ref.iters
    assert r.stats["deflations"] == ref.deflations
    assert r.stats["reorth_second_passes"] >= 1
    np.testing.assert_allclose(r.eigvals, np.linalg.eigvalsh(A)[:4], rtol=1e-12)


def test_rank_deficient_pivot_is_repaired(torch, bbl):
    note("rank-deficient pivot")
    H = synthgen.generate(4000, 400, 20, 0.7, 4)
    lam = np.linalg.eigvalsh(H.to_dense())
    P = synthgen.gaussian_block(H.n, 4, 1)
    P[:, 3] = P[:, 0]  # duplicated column
    r = bbl.block_lanczos(bbl.DeviceCSR.from_host(H, "float64"), dev(torch, P), 4, 1e-9, m_max=300)
    assert r.converged and r.stats["deflations"] >= 1
    np.testing.assert_allclose(r.eigvals, lam[:4], rtol=1e-10)


def test_krylov_exhaustion(torch, bbl):
    note("Krylov exhaustion n=40 b=4")
    H = synthgen.generate(40, 20, 6, 0.7, 2)
    lam = np.linalg.eigvalsh(H.to_dense())
    r = bbl.block_lanczos(bbl.DeviceCSR.from_host(H, "float64"),
                          dev(torch, synthgen.gaussian_block(40, 4, 1)), 16, 1e-300, m_max=10)
    np.testing.assert_allclose(r.eigvals, lam[:16], rtol=0, atol=1e-11 * abs(lam).max())


def test_block_size_one(torch, bbl):
    note("block size 1 (single-vector method)")
    H = synthgen.generate(2000, 400, 20, 0.7, 9)
    lam = np.linalg.eigvalsh(H.to_dense())
    r = bbl.block_lanczos(bbl.DeviceCSR.from_host(H, "float64"),
                          dev(torch, synthgen.gaussian_block(H.n, 1, 2)), 3, 1e-9, m_max=1000)
    assert r.converged
    np.testing.assert_allclose(r.eigvals, lam[:3], rtol=1e-10)


def test_not_converged_reports_current_pairs(torch, bbl):
    note("block cap reached")
    H = synthgen.generate(20000, 400, 20, 0.7, 0)
    r = bbl.block_lanczos(bbl.DeviceCSR.from_host(H, "float64"),
                          dev(torch, synthgen.gaussian_block(H.n, 4, 1)), 4, 1e-10, m_max=5)
    assert r.status == bbl.BBL_E_NOT_CONVERGED and r.stats["iters"] == 5
    assert np.all(np.isfinite(r.eigvals)) and np.all(r.residuals > 0)


def test_breakdown_raised_before_a_redo_is_still_reported(torch, bbl):
    """The QR of block 5 loses rank beyond repair and block 6 needs the second
    Gram-Schmidt sweep (both forced from the host); no check reads the sticky
    breakdown flag before block 6 is redone (checks every 50 blocks), so the
    redo must keep the flag block 5 raised and the solve must fail."""
    note("forced breakdown followed by a redo")
    H = synthgen.generate(4000, 400, 20, 0.7, 4)
    Hd = bbl.DeviceCSR.from_host(H, "float64")
    P = dev(torch, synthgen.gaussian_block(H.n, 4, 1))
    ok = bbl.block_lanczos(Hd, P, 4, 1e-9, m_max=300, check_every=50)
    assert ok.converged and ok.stats["iters"] > 52
    with pytest.raises(bbl.BblError) as e:
        bbl.block_lanczos(Hd, P, 4, 1e-9, m_max=300, check_every=50, fault_block=6)
    assert e.value.code == bbl.BBL_E_BREAKDOWN
    # the default check schedule reports it as well
    with pytest.raises(bbl.BblError) as e:
        bbl.block_lanczos(Hd, P, 4, 1e-9, m_max=300, fault_block=6)
    assert e.value.code == bbl.BBL_E_BREAKDOWN
    # the pooled check stream is healthy after the failures
    again = bbl.block_lanczos(Hd, P, 4, 1e-9, m_max=300, check_every=50)
    assert np.array_equal(again.eigvals, ok.eigvals)


def test_phase_timing_fills_the_stats_and_changes_nothing(torch, bbl):
    note("BBL_FLAG_TIME_PHASES")
    w = synthgen.WORKLOADS["small_fp64_n2e4"]
    H = w.generate()
    Hd = bbl.DeviceCSR.from_host(H, "float64")
    P = bbl.random_pivot(H.n, 4, synthgen.pivot_key(3))
    a = bbl.block_lanczos(Hd, P, 4, 1e-8, m_max=300)
    t = bbl.block_lanczos(Hd, P, 4, 1e-8, m_max=300, time_phases=True)
    assert np.array_equal(a.eigvals, t.eigvals) and a.stats["iters"] == t.stats["iters"]
    for f in ("t_threeterm_ms", "t_reorth_ms", "t_qr_ms", "t_restart_ms", "t_eig_ms"):
        assert a.stats[f] == 0.0
    s = t.stats
    assert s["iters"] <= s["spmm_timed"] <= s["iters"] + CHECK_LAG
    for f in ("spmm_ms", "t_threeterm_ms", "t_reorth_ms", "t_qr_ms", "t_eig_ms"):
        assert s[f] > 0.0, f
    assert s["spmm_ms"] + s["t_threeterm_ms"] + s["t_reorth_ms"] + s["t_qr_ms"] < s["t_total_ms"]
    assert s["t_pivot_ms"] == 0.0 and s["pivot_spmm_calls"] == 0 and s["restarts"] == 0
    # pivot calls report their own time and products
    _, ps = bbl.bootstrap_pivot(Hd, w.n_trunc, 4, 1e-8, m_max=300)
    assert ps["t_pivot_ms"] > 0 and ps["pivot_spmm_calls"] == ps["spmm_calls"] > 0


def test_pivot_overlap_matches_host_svd(torch, bbl):
    """Principal-angle cosines and captured weights against numpy's SVD of
    X^T Q, Q an orthonormal basis of span(P); also for a rank-deficient P
    (a duplicated column) and for X inside span(P) (all cosines 1)."""
    note("pivot overlap diagnostic")
    rng = np.random.default_rng(5)
    n = 30011
    X, _ = np.linalg.qr(rng.standard_normal((n, 10)))
    for case in ("random", "dup", "inside"):
        if case == "inside":
            P = X[:, :8] @ rng.standard_normal((8, 8))
            Xc = X[:, :6].copy()
        else:
            P = rng.standard_normal((n, 8)) + 3.0 * X[:, :8]
            if case == "dup":
                P[:, 7] = P[:, 2]
            Xc = X
        cos, cap = bbl.pivot_overlap(dev(torch, Xc), dev(torch, P))
        U, sv, _ = np.linalg.svd(P, full_matrices=False)
        Q = U[:, sv > 1e-10 * sv[0]]
        ref = np.linalg.svd(Xc.T @ Q, compute_uv=False)
        ref = np.concatenate([ref, np.zeros(Xc.shape[1] - len(ref))])
        # squared cosines are the eigenvalues the kernel computes (a zero one
        # comes out as rounding noise whose square root is ~1e-8)
        np.testing.assert_allclose(cos ** 2, ref ** 2, rtol=0, atol=1e-11)
        assert np.all(np.diff(cos) <= 0)
        np.testing.assert_allclose(cap, np.sum((Xc.T @ Q) ** 2, axis=1), rtol=0, atol=1e-11)
        if case == "inside":
            np.testing.assert_allclose(cos, 1.0, atol=1e-9)


# ----------------------------------------------------------- thick restart
@pytest.mark.parametrize("seed,b,keep,m_max", [(6, 4, 8, 8), (7, 4, 12, 10), (8, 2, 6, 12)])
def test_thick_restart_matches_oracle_and_dense(torch, bbl, seed, b, keep, m_max):
    """FP64: a basis capped at m_max blocks forces many restarts; eigenvalues
    within 1e-10 of numpy's dense eigensolver and of the oracle's restarted
    solve, explicit residuals recomputed on the host, and the final cycle's
    stored basis satisfies V^T V = I and V^T H V = T (its band matrix)."""
    note("thick restart n=1600 b=%d keep=%d m_max=%d" % (b, keep, m_max))
    H = synthgen.generate(1600, 400, 20, 0.7, seed)
    lam = np.linalg.eigvalsh(H.to_dense())
    P = synthgen.gaussian_block(H.n, b, seed)
    Hd = bbl.DeviceCSR.from_host(H, "float64")
    r = bbl.block_lanczos(Hd, dev(torch, P), 4, 1e-10, m_max=m_max, restart_keep=keep)
    ro = oracle.block_lanczos_restarted(H, P, 4, 1e-10, m_max, keep)
    assert r.converged and ro.converged
    assert r.stats["restarts"] >= 5, r.stats
    np.testing.assert_allclose(r.eigvals, lam[:4], rtol=1e-10)
    np.testing.assert_allclose(r.eigvals, ro.eigvals, rtol=1e-10)
    X = r.eigvecs.cpu().numpy()
    res = oracle.ritz_residuals(H, X, r.eigvals)
    assert np.all(res <= 1e-10 * r.stats["hnorm_est"])
    # restarts happen at the same cycle boundaries; the check schedule may
    # end the last cycle a few blocks apart
    assert abs(r.stats["restarts"] - ro.restarts) <= 1, (r.stats["restarts"], ro.restarts)
    m = r.stats["basis_blocks"]
    assert keep // b < m <= m_max
    basis, band = bbl.workspace_views(r.workspace, H.n, b, 4, m_max, bbl.BBL_F64, keep)
    ws = r.workspace
    off = basis - ws.data_ptr()
    V = ws[off:off + m * H.n * b * 8].view(torch.float64).view(m, H.n, b).cpu().numpy()
    Q = np.concatenate([V[j] for j in range(m)], axis=1)
    boff = band - ws.data_ptr()
    bd = ws[boff:boff + m * b * (b + 1) * 8].view(torch.float64).view(m * b, b + 1).cpu().numpy()
    T = np.zeros((m * b, m * b))
    for i in range(m * b):
        for d in range(min(b, i) + 1):
            T[i, i - d] = T[i - d, i] = bd[i, d]
    hn = r.stats["hnorm_est"]
    assert np.max(np.abs(Q.T @ Q - np.eye(m * b))) <= 1e-12
    assert np.max(np.abs(Q.T @ oracle.spmm(H, Q) - T)) <= 1e-10 * hn


def test_fp64_sixteen_vector_solve_matches_oracle_and_dense(torch, bbl):
    """b = 16 in FP64 (values, basis and every product on the matrix-core
    kernels for 16-wide blocks): eigenvalues against the oracle on the same
    pivot and against a dense eigensolve at 1e-10, residuals on the host."""
    note("FP64 b=16 solve vs oracle")
    H = synthgen.generate(3000, 300, 20, 0.7, 21)
    P = synthgen.gaussian_block(3000, 16, 5)
    r = bbl.block_lanczos(bbl.DeviceCSR.from_host(H, "float64"), dev(torch, P), 10, 1e-10,
                          m_max=120, check_every=1)
    ro = oracle.block_lanczos(H, P, 10, 1e-10, 120)
    lam = np.linalg.eigvalsh(H.to_dense())[:10]
    assert r.converged and ro.converged
    np.testing.assert_allclose(r.eigvals, ro.eigvals, rtol=1e-10)
    np.testing.assert_allclose(r.eigvals, lam, rtol=1e-10)
    res = oracle.ritz_residuals(H, r.eigvecs.cpu().numpy(), r.eigvals)
    assert np.all(res <= 1e-10 * r.stats["hnorm_est"]), res / r.stats["hnorm_est"]


def test_thick_restart_fp32_planned_sixteen_vectors(torch, bbl):
    """The C3 shape in small: FP32 values and basis, b = 16 through the
    planned SpMM, k = 10, 12 stored blocks with 32 Ritz vectors kept."""
    note("thick restart FP32 planned b=16 keep=32 m_max=12")
    H = synthgen.generate(40000, 1000, 105, 0.7, 2)
    Hp = bbl.DeviceCSR.from_host(H, "float32", block_rows=1000)
    plan = bbl.spmm_plan(Hp, 16)
    P = bbl.random_pivot(H.n, 16, synthgen.pivot_key(3))
    r = bbl.block_lanczos(Hp, P, 10, 1e-6, m_max=12, restart_keep=32, spmm_plan=plan,
                          time_phases=True)
    assert r.converged and r.stats["restarts"] >= 2, r.stats
    assert r.stats["t_restart_ms"] > 0
    H32 = H.as_float32_values()
    Pref = oracle.bootstrap_pivot(H32, 4000, 8)
    ro = oracle.block_lanczos(H32, Pref, 10, 1e-6, 200)
    np.testing.assert_allclose(r.eigvals, ro.eigvals, rtol=1e-5)
    res = oracle.ritz_residuals(H32, r.eigvecs.cpu().numpy(), r.eigvals)
    assert np.all(res <= 1e-6 * r.stats["hnorm_est"]), res / r.stats["hnorm_est"]


def test_thick_restart_bootstrap_pivot_and_restart_cap(torch, bbl):
    """The pivot's truncated solve restarts too (its pair count raises the
    kept vectors), and a solve out of restarts reports its current pairs
    with their true residuals."""
    note("thick restart in the bootstrap pivot; restart cap")
    w = synthgen.WORKLOADS["small_fp64_n2e4"]
    H = w.generate()
    Hd = bbl.DeviceCSR.from_host(H, "float64")
    P, ps = bbl.bootstrap_pivot(Hd, w.n_trunc, 4, 1e-10, m_max=10, restart_keep=4)
    assert ps["converged"] == 1 and ps["restarts"] >= 1
    Pref = oracle.bootstrap_pivot(H, w.n_trunc, 4)
    sv = np.linalg.svd(Pref.T @ P.cpu().numpy(), compute_uv=False)
    assert sv.min() > 1 - 1e-9
    r = bbl.block_lanczos(Hd, P, 4, 1e-8, m_max=12, restart_keep=8, max_restarts=2)
    assert r.status == bbl.BBL_E_NOT_CONVERGED and r.stats["restarts"] == 2
    X = r.eigvecs.cpu().numpy()
    np.testing.assert_allclose(r.residuals, oracle.ritz_residuals(H, X, r.eigvals), rtol=1e-6)
    ro = bbl.block_lanczos(Hd, P, 4, 1e-8, m_max=12, restart_keep=8)
    assert ro.converged
    np.testing.assert_allclose(ro.eigvals, oracle.block_lanczos(H, Pref, 4, 1e-8, 200).eigvals,
                               rtol=1e-10)


def test_thirty_two_wanted_pairs(torch, bbl):
    """k = 32, the largest pair count: the check's results fill slots 0..64
    of its result area, which must not reach the breakdown-flag copy."""
    note("k=32 wanted pairs")
    H = synthgen.generate(3000, 300, 12, 0.7, 21)
    lam = np.linalg.eigvalsh(H.to_dense())
    Hd = bbl.DeviceCSR.from_host(H, "float64")
    r = bbl.block_lanczos(Hd, dev(torch, synthgen.gaussian_block(H.n, 8, 4)), 32, 1e-9,
                          m_max=300)
    assert r.converged
    np.testing.assert_allclose(r.eigvals, lam[:32], rtol=1e-10)
    f = bbl.pivot_features(Hd, 600, 300, 1e-9, m_max=300, feature_vectors=32)
    assert f["stats"]["converged"] == 1

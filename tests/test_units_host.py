"""Host checks of the LDS-staged unit plan (csrc/sfk_units.h), compiled with g++:
the plan's invariants, and a replay of the staged product with the kernel's
indexing (staged block of double2 slots, one zero row after it, byte offsets
>> 4 plus the lane's pair index, lane groups on their segment ranges) against
the row-by-slice sums of the operator itself."""
import ctypes
import pathlib
import shutil
import subprocess

import numpy as np
import pytest
import scipy.sparse as sp

ROOT = pathlib.Path(__file__).resolve().parents[1]
CSRC = ROOT / "paper_2605_22281_amd" / "csrc"
PADOFF = 0x7FFFFF00
SEG_ALIGN = 4

WRAPPER = r"""
#include "sfk_units.h"
#include <cstring>
extern "C" int plan_c(int NS, const int *sbeg, const int *seg, const int *off, long long nrec,
                      int cols, int rowbytes, int padoff, int cap, int nzcap, int ng, int nbw, int sw,
                      long long *counts, int *unit, int *stage, int *split, int *upart, int *noff,
                      int *group, int *endslot, int *meta, int *grp) {
  sfk::UnitPlan P;
  if (!sfk::plan_units(NS, sbeg, seg, off, nrec, cols, rowbytes, padoff, cap, nzcap, ng, nbw, sw, P))
    return 0;
  counts[0] = (long long)P.unit.size() / 4;
  counts[1] = (long long)P.stage.size();
  counts[2] = (long long)P.split.size();
  counts[3] = (long long)P.upart.size();
  counts[4] = P.nonzeros;
  counts[5] = P.staged;
  std::memcpy(unit, P.unit.data(), sizeof(int) * P.unit.size());
  std::memcpy(stage, P.stage.data(), sizeof(int) * P.stage.size());
  std::memcpy(split, P.split.data(), sizeof(int) * P.split.size());
  std::memcpy(upart, P.upart.data(), sizeof(int) * P.upart.size());
  std::memcpy(noff, P.off.data(), sizeof(int) * P.off.size());
  std::memcpy(group, P.group.data(), sizeof(int) * P.group.size());
  std::memcpy(endslot, P.endslot.data(), sizeof(int) * P.endslot.size());
  std::vector<int> m, g;
  sfk::unit_tables(P, seg, ng, m, g);
  std::memcpy(meta, m.data(), sizeof(int) * m.size());
  std::memcpy(grp, g.data(), sizeof(int) * g.size());
  return 1;
}
"""


@pytest.fixture(scope="module")
def planner(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    d = tmp_path_factory.mktemp("units")
    src = d / "plan.cpp"
    src.write_text(WRAPPER)
    so = d / "plan.so"
    subprocess.run(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-I", str(CSRC), str(src),
                    "-o", str(so)], check=True)
    lib = ctypes.CDLL(str(so))
    lib.plan_c.restype = ctypes.c_int
    return lib


def sliced_copy(M, NS, rowbytes):
    """The column-sliced layout the device builds: slices cols[q * cols / NS ..),
    slice-major segments (rows ascending), each padded to a multiple of 4 records
    (value 0, offset PADOFF), partial slots numbered row by row in slice order."""
    M = sp.csr_matrix(M)
    M.sort_indices()
    rows, cols = M.shape
    cb = [q * cols // NS for q in range(NS + 1)]
    per_slice = [[] for _ in range(NS)]
    nslot = 0
    for i in range(rows):
        c = M.indices[M.indptr[i]:M.indptr[i + 1]]
        v = M.data[M.indptr[i]:M.indptr[i + 1]]
        for s in range(NS):
            m = (c >= cb[s]) & (c < cb[s + 1])
            if m.any():
                per_slice[s].append((i, c[m], v[m], nslot))
                nslot += 1
    seg, off, val, sbeg = [], [], [], [0]
    for s in range(NS):
        for (i, c, v, slot) in per_slice[s]:
            n = len(c)
            npad = -(-n // SEG_ALIGN) * SEG_ALIGN
            p0 = len(off)
            off.extend(list(c * rowbytes) + [PADOFF] * (npad - n))
            val.extend(list(v) + [0.0] * (npad - n))
            seg.append((i, p0, p0 + npad, slot))
        sbeg.append(len(seg))
    off.extend([0] * 256)              # tail padding of the device copy
    val.extend([0.0] * 256)
    return (np.array(sbeg, np.int32), np.array(seg, np.int32).reshape(-1, 4),
            np.array(off, np.int32), np.array(val), nslot, cb)


def run_plan(lib, sbeg, seg, off, cols, rowbytes, cap, ng, nbw, sw=2, nzcap=1 << 30):
    NS = len(sbeg) - 1
    nseg, nrec = len(seg), len(off)
    counts = np.zeros(6, np.int64)
    unit = np.zeros(4 * max(nseg, 1), np.int32)
    stage = np.zeros(max(nseg * cap, 1), np.int32)
    split = np.zeros((ng + 1) * max(nseg, 1), np.int32)
    upart = np.zeros(NS * (nbw + 1), np.int32)
    noff = np.zeros(max(nrec, 1), np.int32)
    group = np.zeros(4 * ng * max(nseg, 1), np.int32)
    endslot = np.zeros(max(nrec, 1), np.int32)
    meta = np.zeros(2 * max(nseg, 1), np.int32)
    grp = np.zeros(2 * ng * max(nseg, 1), np.int32)
    p = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    seg_c = np.ascontiguousarray(seg, np.int32)
    ok = lib.plan_c(NS, p(sbeg), p(seg_c), p(off), ctypes.c_longlong(nrec), cols, rowbytes, PADOFF,
                    cap, nzcap, ng, nbw, sw, p(counts), p(unit), p(stage), p(split), p(upart), p(noff),
                    p(group), p(endslot), p(meta), p(grp))
    if not ok:
        return None
    nu = int(counts[0])
    return dict(unit=unit[:4 * nu].reshape(nu, 4), stage=stage[:counts[1]],
                split=split[:counts[2]].reshape(nu, ng + 1), upart=upart[:counts[3]].reshape(NS, nbw + 1),
                off=noff[:nrec], nonzeros=int(counts[4]), staged=int(counts[5]),
                group=group[:4 * ng * nu].reshape(nu, ng, 4), endslot=endslot[:nrec],
                meta=meta[:2 * nu].reshape(nu, 2), grp=grp[:2 * ng * nu].reshape(nu, ng, 2))


def replay(plan, seg, val, X, RS, cap, ng, nslot):
    """The kernel's staged product, from the tables it reads: per unit, the
    staged block (double2 slots t = row * LPR + pair, rows from the unit's
    padded list, -1 = no row) and a zero row after it, the unit's records
    (meta: first record, count) and each group's range relative to them; lane
    li of a group reads slot (off >> 4) + li; a group streams its records in
    blocks of 4 and stores its sums where a block's last record names a slot."""
    LPR = RS // 2
    capE = cap * RS * 8 // 16
    part = np.full((nslot, RS), np.nan)
    Xp = X.reshape(X.shape[0], LPR, 2)
    for u in range(len(plan["unit"])):
        xs = np.full((capE + LPR, 2), np.nan)
        rows = plan["stage"][u * cap:(u + 1) * cap]
        live = rows >= 0
        xs[:cap * LPR].reshape(cap, LPR, 2)[live] = Xp[rows[live]]
        xs[capE:] = 0.0
        r0, nrec = plan["meta"][u]
        z_off = plan["off"][r0:r0 + nrec]
        z_val = val[r0:r0 + nrec]
        z_end = plan["endslot"][r0:r0 + nrec]
        for g in range(ng):
            rec, rend = plan["grp"][u, g]
            acc = np.zeros((LPR, 2))
            assert (rend - rec) % SEG_ALIGN == 0 and 0 <= rec <= rend <= nrec
            for e0 in range(rec, rend, SEG_ALIGN):
                for e in range(e0, e0 + SEG_ALIGN):
                    o = (min(int(z_off[e]) & 0xFFFFFFFF, cap * RS * 8) & ~15)
                    acc += z_val[e] * xs[(o >> 4) + np.arange(LPR)]
                es = z_end[e0 + SEG_ALIGN - 1]
                if es >= 0:
                    part[es] = acc.reshape(-1)
                    acc = np.zeros((LPR, 2))
    return part


def direct_partials(M, cb, X, nslot):
    M = sp.csr_matrix(M)
    M.sort_indices()
    out = []
    for i in range(M.shape[0]):
        c = M.indices[M.indptr[i]:M.indptr[i + 1]]
        v = M.data[M.indptr[i]:M.indptr[i + 1]]
        for s in range(len(cb) - 1):
            m = (c >= cb[s]) & (c < cb[s + 1])
            if m.any():
                out.append(v[m] @ X[c[m]])
    assert len(out) == nslot
    return np.array(out)


def check_invariants(plan, sbeg, seg, off, cols, rowbytes, cap, ng, nbw, nzcap=1 << 30):
    NS = len(sbeg) - 1
    unit, stage, split, upart, noff = (plan[k] for k in ("unit", "stage", "split", "upart", "off"))
    nu = len(unit)
    # units tile every slice's segments in order; each stays inside one slice
    u = 0
    for s in range(NS):
        assert upart[s, 0] == u and upart[s, -1] >= u
        q = sbeg[s]
        while q < sbeg[s + 1]:
            assert unit[u, 0] == q and unit[u, 1] > q and unit[u, 1] <= sbeg[s + 1]
            q = unit[u, 1]
            u += 1
        assert upart[s, -1] == u
        assert np.all(np.diff(upart[s]) >= 0)
    assert u == nu
    # staged rows: contiguous per unit, at most cap, distinct, every record maps to its column
    assert np.array_equal(unit[:, 2], np.arange(nu) * cap)
    assert np.all(unit[:, 3] >= 1) and np.all(unit[:, 3] <= cap)
    for _, _, z, w in unit:
        assert np.all(stage[z + w:z + cap] == -1) and np.all(stage[z:z + w] >= 0)
    zero = cap * rowbytes
    in_seg = np.zeros(len(off), bool)
    for a, b, z, w in unit:
        rows_u = stage[z:z + w]
        assert len(set(rows_u.tolist())) == w
        for q in range(a, b):
            e0, e1 = seg[q, 1], seg[q, 2]
            in_seg[e0:e1] = True
            real = off[e0:e1] != PADOFF
            assert np.all(noff[e0:e1][~real] == zero)
            slots = noff[e0:e1][real] // rowbytes
            assert np.all(noff[e0:e1][real] % rowbytes == 0) and np.all(slots < w)
            assert np.array_equal(rows_u[slots], off[e0:e1][real] // rowbytes)
    assert np.all(noff[~in_seg] == zero)
    # lane-group ranges: monotone, from the unit's first to its end segment
    for (a, b, _, _), sp_u, gr in zip(unit, split, plan["group"]):
        assert sp_u[0] == a and sp_u[-1] == b and np.all(np.diff(sp_u) >= 0)
        assert seg[b - 1, 2] - seg[a, 1] <= nzcap
        for g in range(ng):
            lo, hi = sp_u[g], sp_u[g + 1]
            want = (lo, hi, seg[lo, 1], seg[hi - 1, 2]) if lo < hi else (0, 0, 0, 0)
            assert tuple(gr[g]) == want
    assert plan["nonzeros"] == int(np.sum(off[:len(off) - 256] != PADOFF))
    # segment ends: exactly the last record of every segment carries its slot
    want = np.full(len(off), -1)
    want[seg[:, 2] - 1] = seg[:, 3]
    assert np.array_equal(plan["endslot"], want)
    assert plan["staged"] == int(unit[:, 3].sum())


def _operator(rows, cols, band, density, seed):
    """Banded random pattern (nearby rows read nearby columns), like a
    projector in a pixel-tile order."""
    rng = np.random.default_rng(seed)
    r, c = [], []
    for i in range(rows):
        centre = int(i * cols / rows)
        lo, hi = max(0, centre - band), min(cols, centre + band)
        cand = np.arange(lo, hi)
        pick = cand[rng.random(len(cand)) < density]
        r.extend([i] * len(pick))
        c.extend(pick.tolist())
    v = rng.standard_normal(len(r))
    return sp.csr_matrix((v, (r, c)), shape=(rows, cols))


@pytest.mark.parametrize("RS,cap,ng,nbw,NS", [(32, 40, 32, 4, 8), (8, 64, 128, 3, 8),
                                              (64, 40, 16, 2, 16), (16, 100, 64, 5, 8)])
def test_plan_invariants_and_replay(planner, RS, cap, ng, nbw, NS):
    M = _operator(300, 960, 18, 0.5, seed=RS + cap)
    rowbytes = RS * 8
    sbeg, seg, off, val, nslot, cb = sliced_copy(M, NS, rowbytes)
    plan = run_plan(planner, sbeg, seg, off, M.shape[1], rowbytes, cap, ng, nbw)
    assert plan is not None
    check_invariants(plan, sbeg, seg, off, M.shape[1], rowbytes, cap, ng, nbw)
    assert len(plan["unit"]) > NS                  # several units per slice at this cap
    X = np.random.default_rng(3).standard_normal((M.shape[1], RS))
    part = replay(plan, seg, val, X, RS, cap, ng, nslot)
    ref = direct_partials(M, cb, X, nslot)
    assert np.allclose(part, ref, rtol=1e-13, atol=1e-13 * np.abs(ref).max())


def test_plan_rejects_segment_wider_than_block(planner):
    M = _operator(60, 400, 200, 0.9, seed=5)        # rows with > cap nonzeros in one slice
    sbeg, seg, off, val, nslot, cb = sliced_copy(M, 8, 256)
    assert run_plan(planner, sbeg, seg, off, 400, 256, 16, 32, 4) is None
    # the same operator fits a block of 64 rows
    plan = run_plan(planner, sbeg, seg, off, 400, 256, 64, 32, 4)
    assert plan is not None
    check_invariants(plan, sbeg, seg, off, 400, 256, 64, 32, 4)


def test_plan_rejects_offsets_outside_the_block(planner):
    M = _operator(40, 64, 8, 0.6, seed=6)
    sbeg, seg, off, val, nslot, cb = sliced_copy(M, 8, 256)
    bad = off.copy()
    bad[seg[3, 1]] = 64 * 256                       # column == cols
    assert run_plan(planner, sbeg, seg, bad, 64, 256, 32, 32, 4) is None
    bad = off.copy()
    bad[seg[2, 1]] = 3 * 256 + 8                    # not a row start
    assert run_plan(planner, sbeg, seg, bad, 64, 256, 32, 32, 4) is None


def test_plan_balances_lane_groups(planner):
    # equal segments: the group ranges differ by at most one segment
    rows, cols = 256, 64
    M = sp.csr_matrix(np.kron(np.eye(8), np.ones((32, 8))))
    sbeg, seg, off, val, nslot, cb = sliced_copy(M, 8, 256)
    plan = run_plan(planner, sbeg, seg, off, cols, 256, 256, 8, 2)
    for sp_u in plan["split"]:
        d = np.diff(sp_u)
        assert d.max() - d.min() <= 1


def test_plan_record_cap(planner):
    M = _operator(300, 960, 18, 0.5, seed=9)
    sbeg, seg, off, val, nslot, cb = sliced_copy(M, 8, 256)
    for nzcap in (64, 200):
        plan = run_plan(planner, sbeg, seg, off, 960, 256, 200, 32, 4, nzcap=nzcap)
        assert plan is not None
        check_invariants(plan, sbeg, seg, off, 960, 256, 200, 32, 4, nzcap=nzcap)
        X = np.random.default_rng(4).standard_normal((960, 32))
        part = replay(plan, seg, val, X, 32, 200, 32, nslot)
        ref = direct_partials(M, cb, X, nslot)
        assert np.allclose(part, ref, rtol=1e-13, atol=1e-13 * np.abs(ref).max())
    # a segment longer than the record cap cannot be planned
    assert run_plan(planner, sbeg, seg, off, 960, 256, 200, 32, 4, nzcap=8) is None

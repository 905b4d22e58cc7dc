"""Batched persistent launch: bitwise equal to per-object launches of the
same dtype; captured HIP graph replays; autotuned shapes."""
import json
import os

import numpy as np
import pytest
import torch

import oracle
import paper_2602_20063_amd as shm
import workloads
from parity import check_value_grad

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def build_batch(n_obj, seed, dtype=np.float32, qscale=1.0):
    r = np.random.default_rng(seed)
    spec = workloads.uneven_batch(r, n_obj=n_obj, mu=6.0 * qscale, sigma=1.0, qmin=1, qmax=5000, Lmax=6)
    luts, objs, off, qb = [], [], 0, 0
    for o in range(n_obj):
        N = int(min(spec["N"][o], 64))
        lut = workloads.random_lut(N, r)
        luts.append(lut.reshape(-1))
        q = int(spec["Q"][o])
        objs.append((off, N, qb, q))
        off += lut.size
        qb += q
    flat = np.concatenate(luts).astype(dtype)
    dirs = workloads.uniform_dirs(qb, r)
    return flat, objs, dirs


@pytest.mark.parametrize("dt,layout", [(torch.float32, 0), (torch.float16, 0), (torch.float16, 1), (torch.float32, 1)])
def test_plan_equals_per_object(dt, layout):
    flat, objs, dirs = build_batch(40, 5)
    code = shm.SHM_F16 if dt == torch.float16 else shm.SHM_F32
    lut_t = torch.as_tensor(flat).to(DEV, dt)
    if layout == shm.SHM_LAYOUT_CELL:  # convert each object to cells
        parts, cobjs, off = [], [], 0
        for (o_off, N, qb, q) in objs:
            n = 6 * (N + 2) * (N + 2) * 4
            cl = shm.to_cells(lut_t[o_off:o_off + n].reshape(1, 6, N + 2, N + 2, 4)).reshape(-1)
            parts.append(cl)
            cobjs.append((off, N, qb, q))
            off += cl.numel()
        lut_t = torch.cat(parts)
        objs = cobjs
    d_t = torch.as_tensor(dirs).to(DEV)
    out = torch.full((dirs.shape[0], 4), float("nan"), device=DEV)
    plan = shm.Plan(objs, code, layout)
    plan.launch(lut_t, d_t, out)
    ref = torch.full_like(out, float("nan"))
    for (off, N, qb, q) in objs:
        if q == 0:
            continue
        n = shm.shm_lut_elems(N, layout)
        shm.shm_query_value_grad(lut_t[off:off + n], code, layout, N, 1, d_t[qb:qb + q], q, ref[qb:qb + q])
    torch.cuda.synchronize()
    assert torch.equal(out, ref)
    plan.close()


def test_plan_matches_oracle_and_shapes():
    flat, objs, dirs = build_batch(25, 6)
    lut_t = torch.as_tensor(flat).to(DEV)
    d_t = torch.as_tensor(dirs).to(DEV)
    ref = oracle.query_objects(flat.reshape(-1).astype(np.float64),
                               [o[0] // 4 for o in objs], [o[1] for o in objs], [o[2] for o in objs],
                               [o[3] for o in objs], dirs)
    plan = shm.Plan(objs, shm.SHM_F32)
    # grid_per_cu 0: one workgroup per work item
    for shape in [(64, 1, 64, 1), (256, 2, 512, 8), (512, 4, 2048, 16), (128, 1, 128 * 7, 3), (256, 1, 256, 0),
                  (64, 4, 512, 0)]:
        plan.set_shape(*shape)
        out = torch.full((dirs.shape[0], 4), float("nan"), device=DEV)
        plan.launch(lut_t, d_t, out)
        torch.cuda.synchronize()
        check_value_grad(out.cpu().numpy(), ref, f"shape {shape}")
    plan.close()


@pytest.mark.parametrize("dt,layout", [(torch.float32, 0), (torch.float16, 1)])
def test_plan_normals_and_row_gaps_every_shape(dt, layout):
    """A plan with normal output, objects whose row ranges leave gaps (and
    one with no queries): at every launch form (one and several queries per
    lane, persistent and one workgroup per item, tiles that split objects
    unevenly) every answered row and normal has the bits of a per-object
    launch, and the gap rows keep their sentinel (the stores of idle lanes
    are dropped, not written past an item's last row)."""
    flat, objs0, dirs0 = build_batch(30, 11)
    code = shm.SHM_F16 if dt == torch.float16 else shm.SHM_F32
    lut_t = torch.as_tensor(flat).to(DEV, dt)
    if layout == shm.SHM_LAYOUT_CELL:
        lut_t, objs0 = to_cells_batch(lut_t, objs0)
    r = np.random.default_rng(12)
    # spread the objects' rows apart: a gap of 0..9 rows before each object
    objs, rows, src = [], 0, []
    for (o_off, N, q0, q) in objs0:
        rows += int(r.integers(0, 10))
        objs.append((o_off, N, rows, q))
        src.append((q0, q))
        rows += q
    objs.insert(5, (objs0[0][0], objs0[0][1], rows, 0))  # no queries
    Q = rows + 7
    dirs = np.zeros((Q, 3), np.float32)
    for (o_off, N, q0, q), (s0, sq) in zip([o for o in objs if o[3] > 0], src):
        dirs[q0:q0 + q] = dirs0[s0:s0 + sq]
    d_t = torch.as_tensor(dirs).to(DEV)
    sentinel = -7.0
    ref = torch.full((Q, 4), sentinel, device=DEV)
    rn = torch.full((Q, 3), sentinel, device=DEV)
    for (o_off, N, q0, q) in objs:
        if q == 0:
            continue
        n = shm.shm_lut_elems(N, layout)
        shm.shm_query_value_grad(lut_t[o_off:o_off + n], code, layout, N, 1, d_t[q0:q0 + q], q, ref[q0:q0 + q],
                                 rn[q0:q0 + q])
    plan = shm.Plan(objs, code, layout)
    for shape in [(64, 1, 64, 1), (256, 1, 256, 0), (64, 2, 128, 0), (256, 2, 512, 4), (128, 4, 512, 0),
                  (64, 4, 64 * 4 * 3, 2), (512, 2, 1024, 0)]:
        plan.set_shape(*shape)
        out = torch.full((Q, 4), sentinel, device=DEV)
        nrm = torch.full((Q, 3), sentinel, device=DEV)
        plan.launch(lut_t, d_t, out, nrm)
        torch.cuda.synchronize()
        assert torch.equal(out.view(torch.int32), ref.view(torch.int32)), shape
        assert torch.equal(nrm.view(torch.int32), rn.view(torch.int32)), shape
    plan.close()


def test_set_shape_refuses_bad_shapes():
    """A shape is checked before the work list is rebuilt: block, queries per
    lane, a tile that is no multiple of block * qpt, workgroups per CU
    outside 0..32; the plan keeps its shape and still answers."""
    flat, objs, dirs = build_batch(4, 3)
    plan = shm.Plan(objs, shm.SHM_F32)
    for bad in [(100, 1, 100, 4), (256, 3, 768, 4), (256, 2, 500, 4), (256, 1, 256, -1), (256, 1, 256, 33)]:
        with pytest.raises(shm.ShmError):
            plan.set_shape(*bad)
    out = torch.full((dirs.shape[0], 4), float("nan"), device=DEV)
    plan.launch(torch.as_tensor(flat).to(DEV), torch.as_tensor(dirs).to(DEV), out)
    torch.cuda.synchronize()
    assert torch.isfinite(out).any()
    plan.close()


def test_graph_capture_replays(tmp_path):
    flat, objs, dirs = build_batch(30, 7)
    lut_t = torch.as_tensor(flat).to(DEV, torch.float16)
    d_t = torch.as_tensor(dirs).to(DEV)
    out = torch.zeros((dirs.shape[0], 4), device=DEV)
    plan = shm.Plan(objs, shm.SHM_F16)
    cache = str(tmp_path / "tune.json")
    shape = plan.autotune(lut_t, d_t, out, cache_path=cache)
    assert shape["tile"] % (shape["block"] * shape["qpt"]) == 0
    saved = json.load(open(cache))
    assert len(saved) == 1
    plan2 = shm.Plan(objs, shm.SHM_F16)
    assert plan2.autotune(lut_t, d_t, out, cache_path=cache) == shape
    plan2.close()
    ref = torch.zeros_like(out)
    plan.launch(lut_t, d_t, ref)
    plan.capture_graph(lut_t, d_t, out)
    for rep in range(3):
        out.zero_()
        torch.cuda.synchronize()
        plan.graph_launch()
        torch.cuda.synchronize()
        assert torch.equal(out, ref), rep
    plan.close()


def test_set_shape_waits_for_earlier_launches():
    """A new tile rewrites the work list in place (the plan allocates only at
    creation): launches already issued on two other streams, not yet waited
    for by the caller, still read the old list to the end and give the same
    bits; the work list never outgrows its creation-time capacity."""
    flat, objs, dirs = build_batch(60, 8, qscale=1.3)
    lut_t = torch.as_tensor(flat).to(DEV)
    d_t = torch.as_tensor(dirs).to(DEV)
    plan = shm.Plan(objs, shm.SHM_F32)
    ref = torch.full((dirs.shape[0], 4), float("nan"), device=DEV)
    plan.launch(lut_t, d_t, ref)
    torch.cuda.synchronize()
    n_default = plan.work_items
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    outs = [torch.full_like(ref, float("nan")) for _ in range(3)]
    for k, st in enumerate((s1, s2)):
        st.wait_stream(torch.cuda.current_stream())
        for _ in range(4):
            plan.launch(lut_t, d_t, outs[k], stream=st)
    plan.set_shape(64, 1, 64, 1)  # the smallest tile: the most work items
    assert plan.work_items > n_default
    plan.launch(lut_t, d_t, outs[2])
    plan.set_shape(512, 4, 4096, 8)
    torch.cuda.synchronize()
    for k in range(3):
        assert torch.equal(outs[k], ref), k
    out = torch.full_like(ref, float("nan"))
    plan.launch(lut_t, d_t, out)
    torch.cuda.synchronize()
    assert torch.equal(out, ref)
    plan.close()


def to_cells_batch(lut_t, objs):
    parts, cobjs, off = [], [], 0
    for (o_off, N, qb, q) in objs:
        n = 6 * (N + 2) * (N + 2) * 4
        cl = shm.to_cells(lut_t[o_off:o_off + n].reshape(1, 6, N + 2, N + 2, 4)).reshape(-1)
        parts.append(cl)
        cobjs.append((off, N, qb, q))
        off += cl.numel()
    return torch.cat(parts), cobjs


@pytest.mark.parametrize("dt,layout", [(torch.float32, 0), (torch.float16, 0), (torch.float16, 1), (torch.float32, 1)])
def test_objects_without_plan_equal_per_object(dt, layout):
    """shm_query_objects (descriptors in device memory, no plan): every
    answered row has the bits of a per-object launch, in any descriptor
    order; objects the kernel must skip (N out of range, a misaligned or
    negative LUT offset, a negative q_begin, no queries) leave their rows
    untouched; tiles of 1, 256 and 257 queries and N = 1 included."""
    flat, objs, dirs = build_batch(40, 7)
    r = np.random.default_rng(8)
    code = shm.SHM_F16 if dt == torch.float16 else shm.SHM_F32
    lut_t = torch.as_tensor(flat).to(DEV, dt)
    # tile-boundary counts and N = 1 on top of the lognormal batch
    extra_lut = [workloads.random_lut(1, r), workloads.random_lut(9, r), workloads.random_lut(4, r)]
    off, qb = lut_t.numel(), dirs.shape[0]
    for lut_x, q in zip(extra_lut, (1, 256, 257)):
        objs.append((off, lut_x.shape[-2] - 2, qb, q))
        off += lut_x.size
        qb += q
    lut_t = torch.cat([lut_t] + [torch.as_tensor(x.reshape(-1)).to(DEV, dt) for x in extra_lut])
    dirs = np.concatenate([dirs, workloads.uniform_dirs(qb - dirs.shape[0], r)])
    if layout == shm.SHM_LAYOUT_CELL:
        lut_t, objs = to_cells_batch(lut_t, objs)
    Q = qb
    # objects to skip, each with rows of its own past the answered ones
    al = 8 if (code == shm.SHM_F16 and layout == shm.SHM_LAYOUT_CELL) else 4
    skip = [(0, 0, Q, 5), (0, shm.SHM_MAX_N + 1, Q + 5, 5), (objs[0][0] + al // 2, objs[0][1], Q + 10, 5),
            (-al, objs[0][1], Q + 15, 5), (0, 4, Q + 20, 0)]
    dirs = np.concatenate([dirs, workloads.uniform_dirs(25, r)])
    d_t = torch.as_tensor(dirs).to(DEV)
    order = list(r.permutation(len(objs)))
    descs = [objs[i] for i in order] + skip
    descs.insert(3, (0, objs[0][1], -5, 5))  # negative q_begin: skipped, writes nothing
    sentinel = -7.0
    out = torch.full((Q + 25, 4), sentinel, device=DEV)
    nrm = torch.full((Q + 25, 3), sentinel, device=DEV)
    ws = torch.empty(shm.shm_query_objects_workspace(len(descs)), dtype=torch.uint8, device=DEV)
    shm.shm_query_objects(lut_t, code, layout, shm.objects_tensor(descs, DEV), len(descs), d_t, out, nrm, ws)
    ref = torch.full_like(out, sentinel)
    rn = torch.full_like(nrm, sentinel)
    for (o_off, N, q0, q) in objs:
        n = shm.shm_lut_elems(N, layout)
        shm.shm_query_value_grad(lut_t[o_off:o_off + n], code, layout, N, 1, d_t[q0:q0 + q], q, ref[q0:q0 + q],
                                 rn[q0:q0 + q])
    torch.cuda.synchronize()
    assert torch.equal(out.view(torch.int32), ref.view(torch.int32))
    assert torch.equal(nrm.view(torch.int32), rn.view(torch.int32))
    # the same call again, reusing the workspace: same bits
    out2 = torch.full_like(out, sentinel)
    shm.shm_query_objects(lut_t, code, layout, shm.objects_tensor(descs, DEV), len(descs), d_t, out2, None, ws)
    torch.cuda.synchronize()
    assert torch.equal(out2.view(torch.int32), ref.view(torch.int32))


def test_objects_without_plan_many_small_objects():
    """More objects than the scan has lanes (several per lane), tiny query
    counts and face sizes: the tile offsets and the object search."""
    r = np.random.default_rng(9)
    n_obj = 2500
    Ns = r.integers(1, 7, n_obj)
    qs = r.integers(0, 40, n_obj)
    luts = [workloads.random_lut(int(N), r).reshape(-1) for N in Ns]
    offs = np.concatenate([[0], np.cumsum([x.size for x in luts])[:-1]])
    qb = np.concatenate([[0], np.cumsum(qs)[:-1]])
    objs = [(int(offs[o]), int(Ns[o]), int(qb[o]), int(qs[o])) for o in range(n_obj)]
    lut_t = torch.as_tensor(np.concatenate(luts)).to(DEV)
    Q = int(qs.sum())
    d_t = torch.as_tensor(workloads.uniform_dirs(Q, r)).to(DEV)
    out = shm.query_objects(lut_t, d_t, objs)
    ref = torch.empty_like(out)
    for (o_off, N, q0, q) in objs:
        if q:
            n = shm.shm_lut_elems(N)
            shm.shm_query_value_grad(lut_t[o_off:o_off + n], shm.SHM_F32, 0, N, 1, d_t[q0:q0 + q], q, ref[q0:q0 + q])
    torch.cuda.synchronize()
    assert torch.equal(out.view(torch.int32), ref.view(torch.int32))

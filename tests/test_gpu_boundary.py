"""The C-ABI boundary on the GPU: the caller-supplied workspace of
svds_solve_prepared (the workspace that Section 3.3 lets the library allocate
or the user supply) and concurrent solves on one prepared matrix.

Every test prints the case it runs before touching the GPU."""
import threading

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1607_01404_amd as P
    P.load_library()
    return P


def _same(a, b):
    return all(bool((x.cpu() == y.cpu()).all()) for x, y in zip(a[:4], b[:4]))


CASES = [
    ("banded smallest jacobi b=2 (one-pass product, JD)", "smallest",
     dict(block_size=2, precond=1, seed=3)),
    ("banded smallest block-jacobi b=1 GD+k stage 2", "smallest",
     dict(block_size=1, precond=3, pc_block=32, stage2_solver=0, seed=4, force_stage2=1)),
    ("banded largest mixed b=4", "largest", dict(block_size=4, precision=1, seed=5)),
    ("banded largest normal-equations method", "largest", dict(block_size=1, method=1, seed=6)),
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_workspace_solve_is_bitwise_the_pool_solve(P, case):
    import torch
    name, target, opts = CASES[case]
    A = synth.banded_scaled(3000, 1500, seed=9, log_lo=-3.0)
    normA = float(np.linalg.norm(A.toarray(), 2))
    _say("workspace", name)
    M = P.Matrix.from_scipy(A)
    opts = dict(opts, norm_A=normA, autotune=0)
    nbytes = M.workspace_size(4, target, **opts)
    assert nbytes > 8 * 1500 * 35 * 4  # at least V, W and their restart copies
    ref = M.solve(4, target, 1e-10, **opts)
    assert ref[4]["converged"], ref[4]
    # exactly the reported size, at an offset that is not 256-byte aligned
    ws = torch.empty(nbytes + 8, dtype=torch.uint8, device="cuda")
    view = ws[8:]
    got = M.solve(4, target, 1e-10, workspace=view, **opts)
    assert got[4]["converged"] and got[4]["matvecs"] == ref[4]["matvecs"]
    assert _same(got, ref)
    # one byte short of what the solve needs is rejected before any launch
    with pytest.raises(P.SvdsError) as e:
        M.solve(4, target, 1e-10, workspace=ws[: nbytes - 256 - 1], **opts)
    assert e.value.code == -1
    M.close()


def test_workspace_size_rejects_bad_options(P):
    A = synth.uniform_workload()
    _say("workspace_size argument checks")
    M = P.Matrix.from_scipy(A)
    with pytest.raises(P.SvdsError):
        M.workspace_size(5, "largest", block_size=9)
    with pytest.raises(P.SvdsError):
        M.workspace_size(0, "largest")
    # the smallest values keep the refined factor: more workspace than the largest
    assert M.workspace_size(5, "smallest") > M.workspace_size(5, "largest")
    M.close()


def test_concurrent_solves_with_different_blocks_on_one_matrix(P):
    """Two solves on distinct streams, block sizes 1 and 4, on one prepared
    matrix that neither has tuned yet: each equals, bit for bit, the same
    solve run alone afterwards (the launch shapes the first solves fixed in
    the handle are the ones the later solves use)."""
    import torch
    A = synth.banded_scaled(20000, 10000, seed=12, log_lo=-2.0)
    normA = float(np.linalg.norm(A.toarray(), 2)) if A.shape[1] <= 2000 else None
    _say("concurrent solves b=1 and b=4 on one prepared matrix")
    M = P.Matrix.from_scipy(A)
    kw = dict(norm_A=normA) if normA else {}
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    blocks = [1, 4]
    out = [None, None]
    err = []

    def run(i):
        try:
            torch.cuda.set_device(0)
            out[i] = M.solve(5, "smallest", 1e-10, stream=streams[i], block_size=blocks[i],
                             precond=1, seed=2, **kw)
        except Exception as e:  # noqa: BLE001
            err.append(e)

    th = [threading.Thread(target=run, args=(i,)) for i in range(2)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    assert not err, err
    torch.cuda.synchronize()
    for i in range(2):
        again = M.solve(5, "smallest", 1e-10, block_size=blocks[i], precond=1, seed=2, **kw)
        assert out[i][4]["converged"] and again[4]["converged"]
        assert _same(out[i], again), blocks[i]
    P.stream_release(streams[0])
    P.stream_release(streams[1])
    M.close()

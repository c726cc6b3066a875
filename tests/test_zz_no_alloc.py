"""The entry point for callers that cannot allocate: sgtv_backprojection_noalloc
keeps its intermediate vectors in the library's static device buffer and must
give exactly what sgtv_backprojection gives.  Two calls in a row on different
contexts (the second with a smaller problem, so the shared buffer holds the
first call's larger contents), host and device outputs, and a problem past
the buffer's limit refused with SGTV_ESHAPE."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sg():
    import torch
    assert torch.cuda.is_available()
    from paper_1601_08201_amd import sgtv
    sgtv.lib()
    return sgtv


def reconstructor(sg, cfg, seed):
    from paper_1601_08201_amd import datagen
    prob = datagen.make_problem(cfg, seed)
    R = sg.Reconstructor(device=0)
    R.set_problem(prob)
    return R, prob


def test_noalloc_matches_backprojection_on_two_calls(sg):
    import torch
    R1, p1 = reconstructor(sg, "teflon", 1)      # 19926 hyper-voxels
    R2, p2 = reconstructor(sg, "small", 3)       # 8192 hyper-voxels
    assert p2.J < p1.J
    for R, prob in ((R1, p1), (R2, p2)):
        print("case", prob.meta["cfg"], "J =", prob.J, flush=True)
        want = sg.sgtv_backprojection(R._ctx)
        got = sg.sgtv_backprojection_noalloc(R._ctx)
        np.testing.assert_array_equal(got, want)
        dev = torch.empty(prob.J, dtype=torch.float32, device="cuda")
        sg.sgtv_backprojection_noalloc(R._ctx, out=dev)
        np.testing.assert_array_equal(dev.cpu().numpy(), want)
        assert np.all(want >= 0) and np.any(want > 0)
    R1.close()
    R2.close()


def test_noalloc_refuses_problems_past_its_buffer(sg):
    # one entry per column, column j in row j % 64 (rows sorted, columns ascending)
    J, I = sg.SGTV_NOALLOC_MAX_VOXELS + 4, 64
    col = np.concatenate([np.arange(i, J, I, dtype=np.int32) for i in range(I)])
    rowptr = np.zeros(I + 1, np.int64)
    rowptr[1:] = np.cumsum([len(range(i, J, I)) for i in range(I)])
    R = sg.Reconstructor(device=0)
    R.set_system(I, 1, 2, J // 2, rowptr, col, np.full(col.size, 0.5, np.float32))
    R.set_data(np.full(I, 3.0, np.float32), np.full(I, 0.1, np.float32), 0.1, 1.0, 1)
    with pytest.raises(sg.SgtvError) as ei:
        sg.sgtv_backprojection_noalloc(R._ctx)
    assert ei.value.code == sg.SGTV_ESHAPE
    R.close()

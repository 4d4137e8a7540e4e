"""Per-launch event timing of the step (mhd_set_timing / mhd_get_timing):
launch counts per kernel class over enough steps that the library reads its
event ring before the end (it waits for pending events only once 512 are
recorded), and the state bitwise the same as a run without timing."""
import numpy as np
import pytest

from paper_1608_08748_amd import binding, inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    torch.cuda.set_device(0)


def _box(W):
    box = binding.Box(W.shape[1:], precision=binding.FP64)
    box.init_state(W)
    return box


# launches per step and class (x rows of at most 256 cells): NONADV faces y,
# z, x-rows and the face-field update per substage; the ADV y march and the
# two z-march update launches per substage, which form the x faces
# themselves; the tail of the step; the CFL reduction
PER_STEP = {"setup": 0, "nonadv_face": 9, "nonadv_update": 3, "adv_face": 3, "adv_update": 6, "tail": 1,
            "reduce": 1, "poisson": 0}


def test_timing_counts_and_state():
    W = inputs.c2(n=16)
    a, b = _box(W), _box(W)
    b.set_timing(True)
    K = 30   # 750 launches: the ring is read once on the way
    for _ in range(K):
        a.step_cfl()
        b.step_cfl()
    t = b.get_timing()
    for k, n in PER_STEP.items():
        assert t[k][1] == n * K, (k, t[k])
        assert t[k][0] >= 0.0, (k, t[k])
    assert t["nonadv_face"][0] > 0.0 and t["adv_update"][0] > 0.0
    assert np.array_equal(a.get_state(), b.get_state())
    # the accumulators keep counting after a read; enabling again clears them
    b.step_cfl()
    assert b.get_timing()["reduce"][1] == K + 1
    b.set_timing(True)
    assert all(v == (0.0, 0) for v in b.get_timing().values())
    b.set_timing(False)
    b.step_cfl()
    assert all(v == (0.0, 0) for v in b.get_timing().values())

"""GPU parity of the two-site 2-TDVP generator H^(2) C (SM Eq. S-2TDVP) on
dense operands against the oracle contraction, through the C ABI."""
import numpy as np
import pytest

from oracle import tdvp as otd
from paper_2212_11973_amd import tantrg as T
from paper_2212_11973_amd import workloads as WL

pytestmark = pytest.mark.gpu


def _apply(L, W1, W2, C, R, precision=T.TT_FP64):
    import torch
    assert torch.cuda.is_available()
    dev = torch.device("cuda:0")
    tl, t1, t2, tc, tr = (torch.from_numpy(np.ascontiguousarray(x)).to(dev) for x in (L, W1, W2, C, R))
    out = torch.empty_like(tc)
    Dl, DH, Dr = L.shape[0], L.shape[1], R.shape[0]
    T.tt_heff2_apply(Dl, Dr, DH, tl.data_ptr(), t1.data_ptr(), t2.data_ptr(), tc.data_ptr(), tr.data_ptr(),
                     out.data_ptr(), precision, torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("Dl,Dr,DH,seed", [(1, 1, 1, 0), (3, 5, 2, 1), (16, 16, 4, 2), (40, 24, 6, 3),
                                           (64, 48, 18, 4), (17, 70, 10, 5)])
def test_heff2_matches_oracle(Dl, Dr, DH, seed):
    print("heff2", Dl, Dr, DH, flush=True)
    L, W1, W2, C, R = WL.heff2_inputs(Dl, Dr, DH, seed)
    got = _apply(L, W1, W2, C, R)
    ref = otd.heff2(L, W1, W2, R, C)
    scale = np.abs(ref).max()
    assert np.abs(got - ref).max() <= 1e-12 * scale
    # a second call with the same sizes reuses the plans
    assert np.array_equal(_apply(L, W1, W2, C, R), got)


def test_heff2_after_a_size_change():
    # the cached R2 buffer is reused at a smaller layout: its zero blocks are
    # refilled (entries the GEMM never writes)
    for (Dl, Dr, DH, seed) in [(17, 70, 10, 5), (32, 24, 8, 7), (8, 8, 4, 3), (16, 8, 4, 4)]:
        L, W1, W2, C, R = WL.heff2_inputs(Dl, Dr, DH, seed)
        ref = otd.heff2(L, W1, W2, R, C)
        assert np.abs(_apply(L, W1, W2, C, R) - ref).max() <= 1e-12 * np.abs(ref).max()


def test_heff2_fp32_contractions():
    L, W1, W2, C, R = WL.heff2_inputs(32, 24, 8, 7)
    got = _apply(L, W1, W2, C, R, T.TT_FP32)
    ref = otd.heff2(L, W1, W2, R, C)
    assert np.linalg.norm(got - ref) <= 2e-6 * np.linalg.norm(ref)


def test_heff2_rejects_bad_arguments():
    with pytest.raises(T.TTError):
        T.tt_heff2_apply(0, 4, 2, 1, 1, 1, 1, 1, 1)
    with pytest.raises(T.TTError):
        T.tt_heff2_apply(4, 4, 2, 0, 1, 1, 1, 1, 1)

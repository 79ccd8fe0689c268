"""The Python binding rejects mismatched query tensors before anything reaches
the library (no GPU needed: host tensors stand in for device ones, and every
mismatch below is caught before the device placement is looked at)."""
import pytest

torch = pytest.importorskip("torch")

from paper_1509_06957_amd import mrpt  # noqa: E402


def _ok(nq=5, d=16, k=3):
    return (torch.zeros((nq, d), dtype=torch.float32), torch.zeros((nq, k), dtype=torch.int32),
            torch.zeros((nq, k), dtype=torch.float32))


def test_matching_tensors_pass():
    Q, oi, od = _ok()
    mrpt.check_query_tensors(16, Q, 3, oi, od, torch.zeros(5, dtype=torch.int32))


@pytest.mark.parametrize("bad", ["q_dim", "q_rank", "q_dtype", "idx_shape", "dist_shape", "idx_dtype",
                                 "dist_dtype", "s_short", "s_dtype", "noncontig", "not_tensor"])
def test_each_mismatch_raises(bad):
    Q, oi, od = _ok()
    s = None
    if bad == "q_dim":
        Q = torch.zeros((5, 17))
    elif bad == "q_rank":
        Q = torch.zeros(80)
    elif bad == "q_dtype":
        Q = torch.zeros((5, 16), dtype=torch.float64)
    elif bad == "idx_shape":
        oi = torch.zeros((5, 4), dtype=torch.int32)
    elif bad == "dist_shape":
        od = torch.zeros((4, 3))
    elif bad == "idx_dtype":
        oi = torch.zeros((5, 3), dtype=torch.int64)
    elif bad == "dist_dtype":
        od = torch.zeros((5, 3), dtype=torch.float16)
    elif bad == "s_short":
        s = torch.zeros(4, dtype=torch.int32)
    elif bad == "s_dtype":
        s = torch.zeros(5, dtype=torch.int64)
    elif bad == "noncontig":
        Q = torch.zeros((16, 5)).t()
    elif bad == "not_tensor":
        od = [0.0] * 15
    with pytest.raises((ValueError, TypeError)):
        mrpt.check_query_tensors(16, Q, 3, oi, od, s)


def test_index_query_checks_before_the_library():
    # an Index whose handle was never built: the call must fail in the checks,
    # never reach the library with these tensors
    ix = object.__new__(mrpt.Index)
    ix.handle = None
    ix.info = mrpt.mrpt_index_desc(n=100, d=16, T=2, depth=2)
    Q = torch.zeros((5, 15))
    with pytest.raises(ValueError):
        ix.query(Q, 3, 1)
    Q, oi, od = _ok()
    with pytest.raises(ValueError):
        ix.query(Q, 3, 1, out=(oi[:, :2].contiguous(), od))
    with pytest.raises((ValueError, TypeError)):
        ix.query(Q, 3, 1, s_count=torch.zeros(2, dtype=torch.int32))
    # well-formed host tensors get as far as the device check
    with pytest.raises(TypeError, match="CUDA"):
        ix.query(Q, 3, 1, out=(oi, od))

"""The no-allocation error table (bs_ns_error_table_noalloc) against the
allocating entry point, on two calls in a row, the second with fewer samples."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_error_table_noalloc_matches_allocating_entry_point():
    import torch
    assert torch.cuda.is_available()
    from paper_2406_07366_amd import binding as B
    from paper_2406_07366_amd import ns_mlp
    print("\n[case] error table noalloc vs allocating, n = 200000 then 777", flush=True)
    mlp = B.MLP(B.mlp_init(3))
    X, T, A = ns_mlp.make_dataset(200_000, 9)
    for m in (200_000, 777):
        Xs, Ts, As = X[:m].contiguous(), T[:m].contiguous(), A[:m].contiguous()
        rms, mx = B.ns_error_table(mlp, Xs, Ts, As)
        _, _, nb = B.ns_error_bins()
        r_dev = torch.full((nb,), -1.0, dtype=torch.float32, device="cuda")
        m_dev = torch.full((nb,), -1.0, dtype=torch.float32, device="cuda")
        B.ns_error_table_noalloc(mlp, Xs, Ts, As, r_dev, m_dev)
        torch.cuda.synchronize()
        r2, m2 = r_dev.cpu().numpy(), m_dev.cpu().numpy()
        print(f"  n={m}: rms {rms[:3]} ... noalloc {r2[:3]} ...")
        np.testing.assert_array_equal(r2, rms)
        np.testing.assert_array_equal(m2, mx)
    with pytest.raises(B.BsError):
        big = torch.zeros((300_000, 8), dtype=torch.float32, device="cuda")
        B.ns_error_table_noalloc(mlp, big, big[:, :3].contiguous(),
                                 torch.zeros((300_000, 7), dtype=torch.float64, device="cuda"),
                                 r_dev, m_dev)

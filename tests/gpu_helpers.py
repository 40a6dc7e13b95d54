"""Shared helpers of the GPU tests: device copies of synthetic inputs and the
comparison of one GPU level against the oracle fed the same A_k."""
import numpy as np

from oracle import amg_oracle as O


def to_dev(A):
    import torch
    dev = "cuda"
    return (torch.from_numpy(A.row_ptr).to(dev), torch.from_numpy(A.col).to(dev),
            torch.from_numpy(A.val).to(dev))


def dev_vec(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).to("cuda")


def oracle_level(ex, opts):
    """Run the oracle's loop body on the GPU's exported A_k and B_k."""
    A = O.validate_csr(ex["row_ptr"], ex["col"], ex["val"])
    return O.coarsen_level(A, ex["B"], opts)


def compare_level(ex, lv, nxt=None, tol=1e-12):
    """Bit-exact strength / MIS / aggregates; interpolation and A_{k+1} to tol."""
    assert np.array_equal(ex["strong"].astype(bool), lv.C), "strength mask differs"
    assert np.array_equal(ex["state"].astype(np.int64), lv.s), "MIS(2) state differs"
    assert np.array_equal(ex["agg"].astype(np.int64), lv.agg), "aggregates differ"
    assert np.allclose(ex["pval"], lv.pval, rtol=1e-14, atol=0), "interpolation differs"
    if nxt is not None:
        Ac = lv.Ac
        assert np.array_equal(nxt["row_ptr"], Ac.indptr), "coarse row pointers differ"
        assert np.array_equal(nxt["col"], Ac.indices), "coarse columns differ"
        # per-entry bound relative to the magnitude of the summed terms
        rows = np.repeat(np.arange(lv.n), np.diff(lv.A.indptr))
        mag = np.abs(lv.pval[rows] * lv.A.data * lv.pval[lv.A.indices])
        import scipy.sparse as sp
        M = sp.csr_matrix((mag, (lv.agg[rows], lv.agg[lv.A.indices])), shape=Ac.shape)
        M.sum_duplicates()
        M.sort_indices()
        bound = tol * M.data + 1e-300
        err = np.abs(nxt["val"] - Ac.data)
        assert np.all(err <= bound), f"coarse values differ: max ratio {np.max(err / bound):.3g}"
        fro = np.linalg.norm(nxt["val"] - Ac.data) / np.linalg.norm(Ac.data)
        assert fro <= tol

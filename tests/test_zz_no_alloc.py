"""The batched evaluation entry point that allocates nothing
(pyhea_sro_eval_batch_noalloc) against pyhea_sro_eval_batch, through the C ABI:
two calls in a row sharing the library's fixed device scratch, the second with
a smaller input, on a geometry whose configurations span several workgroups
(partial sums in the scratch) and on one that fits one workgroup each."""
import numpy as np
import pytest

from paper_2411_18906_amd import binding as pb
from paper_2411_18906_amd import workloads as wl

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def problem(lattice, L, M, S, seed):
    rng = np.random.default_rng(seed)
    return wl.Problem(lattice, L, M, S, rng.uniform(-0.2, 0.2, (S, M, M)), np.array([1.0, 0.5, 0.25][:S]),
                      np.zeros(0, np.int8))


def run(fn, p, batch):
    K = batch.shape[0]
    counts = torch.full((K, p.S, p.M, p.M), -7, dtype=torch.int32, device="cuda")
    S_F = torch.full((K, 2), -1.0, dtype=torch.float64, device="cuda")
    fn(p.lattice, p.L, p.M, p.S, batch, counts, p.target, p.weight, S_F)
    torch.cuda.synchronize()
    return counts.cpu().numpy(), S_F.cpu().numpy()


@pytest.mark.parametrize("case", ["fcc20_split", "fcc8_whole", "bcc_gather"])
def test_noalloc_equals_allocating_entry_point_two_calls(case):
    if case == "fcc20_split":
        p, sizes = wl.fcc20_chain(), (6, 3)          # few configurations: each spread over many workgroups
    elif case == "fcc8_whole":
        p, sizes = problem(wl.FCC, (8, 8, 8), 4, 2, 21), (700, 65)
    else:
        p, sizes = problem(wl.BCC, (5, 5, 5), 3, 2, 22), (40, 9)   # odd-Lx BCC
    for K, seed in zip(sizes, (31, 32)):
        batch = torch.from_numpy(wl.iid_configs(p.N, p.M, K, seed=seed)).cuda()
        c_ref, sf_ref = run(pb.pyhea_sro_eval_batch, p, batch)
        c_na, sf_na = run(pb.pyhea_sro_eval_batch_noalloc, p, batch)
        np.testing.assert_array_equal(c_na, c_ref)
        np.testing.assert_array_equal(sf_na, sf_ref)


def test_noalloc_rejects_batches_beyond_its_scratch():
    p = problem(wl.FCC, (4, 4, 4), 4, 2, 23)
    K = 5_000_000          # flags alone: 20 MB > the 16 MiB array
    batch = torch.zeros((K, p.N), dtype=torch.int8, device="cuda")
    counts = torch.zeros((K, p.S, p.M, p.M), dtype=torch.int32, device="cuda")
    with pytest.raises(pb.PyheaError, match="split the batch"):
        pb.pyhea_sro_eval_batch_noalloc(p.lattice, p.L, p.M, p.S, batch, counts)

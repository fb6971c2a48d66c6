"""GPU NPR contraction (sp_npr_path_links + sp_npr_contract, and the fused sp_npr_contract_links) against the
FP64 oracle (oracle/npr.py).

Small lattices are compared whole. On the 20^3x64 workload field, sampled hypercubes are compared with the
oracle run on the hypercube alone: a hypercube's path links and its O_i(z) depend only on the links and
fields at its 16 corners, which form a 2^4 lattice of their own (paths never use a link that leaves the
hypercube, so the wrap-around links of the 2^4 lattice are never read)."""
import numpy as np
import pytest
import torch

import lattice_inputs as li
import paper_1511_00088_amd as sp
from gpu_common import DEV, announce, to_dev, to_host
from oracle import npr

pytestmark = pytest.mark.gpu


def _fields(n, V, seed):
    rng = np.random.default_rng(seed)
    return [rng.standard_normal((n, V, 3)) + 1j * rng.standard_normal((n, V, 3)) for _ in range(4)]


@pytest.mark.parametrize("dims,labels", [
    ((4, 4, 4, 4), (15, 15, 15, 15)),
    ((4, 6, 2, 8), (3, 5, 12, 9)),
    ((6, 4, 4, 2), (0, 0, 0, 0)),
    ((4, 4, 4, 4), (1, 8, 6, 3)),
])
def test_npr_matches_oracle(dims, labels):
    announce(f"npr dims={dims} labels={labels}")
    V = li.volume(dims)
    U = li.near_identity_links(dims, 0.7, 601)
    f = _fields(3, V, 602)
    lat = sp.Lattice(dims)
    uad = sp.npr_path_links(lat, to_dev(U))
    O = sp.npr_contract(lat, uad, *[to_dev(x) for x in f], labels)
    torch.cuda.synchronize()
    P = npr.path_links(dims, U)
    assert np.max(np.abs(to_host(uad) - P)) <= 1e-14
    ref = npr.contract(dims, P, *f, *labels)
    assert np.max(np.abs(to_host(O) - ref)) <= 1e-12 * np.max(np.abs(ref))
    # the fused contraction (path links built in on-chip memory): the same arithmetic in the same order, so the
    # same bits as the two launches
    Of = sp.npr_contract_links(lat, to_dev(U), *[to_dev(x) for x in f], labels)
    assert torch.equal(Of, O)


@pytest.mark.parametrize("n", [1, 4, 5, 9])
def test_npr_fused_field_set_counts(n):
    """Field-set counts around the staging chunk of four (a partial last chunk, exactly one chunk, several)."""
    dims = (4, 6, 2, 8)
    V = li.volume(dims)
    U = li.near_identity_links(dims, 0.7, 611)
    f = _fields(n, V, 612 + n)
    labels = (5, 10, 3, 3)
    lat = sp.Lattice(dims)
    Of = to_host(sp.npr_contract_links(lat, to_dev(U), *[to_dev(x) for x in f], labels))
    ref = npr.contract(dims, npr.path_links(dims, U), *f, *labels)
    assert Of.shape == ref.shape
    assert np.max(np.abs(Of - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_npr_workload_field_sampled_hypercubes():
    c = li.cfg1()
    dims = c["dims"]
    announce(f"npr {dims} sampled")
    V = li.volume(dims)
    U = c["links"]
    f = _fields(2, V, 603)
    labels = (15, 15, 15, 15)
    lat = sp.Lattice(dims)
    uad = sp.npr_path_links(lat, to_dev(U))
    O = to_host(sp.npr_contract(lat, uad, *[to_dev(x) for x in f], labels))
    cs = npr.corner_sites(dims)  # [nz][16]
    zs = np.unique(np.concatenate([np.random.default_rng(604).integers(0, cs.shape[0], 48), [0, cs.shape[0] - 1]]))
    small = (2, 2, 2, 2)
    sites = cs[zs]  # corner A of the hypercube is site A of the 2^4 lattice
    uad_s = to_host(uad[torch.as_tensor(zs, device=DEV)])
    # fused with the path links built on chip: the same bits as the two launches at every hypercube
    Of = to_host(sp.npr_contract_links(lat, to_dev(U), *[to_dev(x) for x in f], labels))
    assert np.array_equal(Of, O)
    for k, z in enumerate(zs):
        Us = U[:, sites[k]]
        P = npr.path_links(small, Us)
        assert np.max(np.abs(uad_s[k] - P[0])) <= 1e-14
        ref = npr.contract(small, P, *[x[:, sites[k]] for x in f], *labels)
        assert np.max(np.abs(O[:, z] - ref[:, 0])) <= 1e-12 * np.max(np.abs(ref))


def test_npr_errors():
    dims = (4, 4, 4, 4)
    lat = sp.Lattice(dims)
    V = li.volume(dims)
    uad = sp.npr_path_links(lat, to_dev(li.haar_links(dims, 605)))
    f = [to_dev(x) for x in _fields(1, V, 606)]
    with pytest.raises(sp.StagError):
        sp.npr_contract(lat, uad, *f, (16, 0, 0, 0))
    with pytest.raises(sp.StagError):
        sp.npr_contract_links(lat, to_dev(li.haar_links(dims, 605)), *f, (0, 0, -1, 0))

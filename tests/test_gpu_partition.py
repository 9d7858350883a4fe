"""The parts of a partition of the elements, each assembled on the GPU as a
mesh of its own, sum to the whole mesh's assembly: the identity a split of
the elements over several GPUs (each summing partial rows, then adding the
rows it shares with the others) rests on, checked here on one GPU."""
import numpy as np
import pytest

import meshgen as mg
import oracle
from tests.helpers import fp64_errors, scatter_part

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1805_03949_amd as fea  # noqa: E402


def _type_sorted_parts(types, parts):
    """Contiguous ranges of the type-sorted element order, equal in element
    count: the cut the static split of the cost-model study makes."""
    perm = np.argsort(types, kind="stable")
    return np.array_split(perm, parts)


@pytest.mark.parametrize("variant", ["rowsym", "rowowner"])
def test_parts_assembled_apart_sum_to_the_whole(variant):
    var = {"rowsym": fea.ROWSYM, "rowowner": fea.ROWOWNER}[variant]
    m = mg.heterogeneous(16, seed=6, brick=4, jitter=0.1)
    print(f"[case] hetero16 seed 6, {variant}, E={m.n_elems}", flush=True)
    dm = fea.DeviceMesh(m, device="cuda:0")
    g = dm.graph()
    v, r, st = dm.assemble(g, use_nh=True, variant=var, precision=fea.FP64, out_dtype=fea.F64)
    torch.cuda.synchronize()
    assert int(st.item()) == -1
    ex = g.export()
    row_ptr, col = ex["row_ptr"].cpu().numpy(), ex["col"].cpu().numpy()
    whole, whole_r = v.cpu().numpy(), r.cpu().numpy()
    acc, accr = np.zeros_like(whole), np.zeros_like(whole_r)
    for elems in _type_sorted_parts(m.types, 8):
        sub, nodes = mg.submesh(m, elems, return_nodes=True)
        sdm = fea.DeviceMesh(sub, device="cuda:0")
        sg = sdm.graph()
        sv, sr, sst = sdm.assemble(sg, use_nh=True, variant=var, precision=fea.FP64, out_dtype=fea.F64)
        torch.cuda.synchronize()
        assert int(sst.item()) == -1
        sx = sg.export()
        scatter_part(row_ptr, col, nodes, sx["row_ptr"].cpu().numpy(), sx["col"].cpu().numpy(),
                     sv.cpu().numpy(), 3, acc, sr.cpu().numpy(), accr)
        sg.destroy()
    ev, er = fp64_errors(acc, whole, row_ptr, 3, accr, whole_r)
    assert ev < 1e-12 and er < 1e-12, (ev, er)
    # and the whole against the oracle
    og = oracle.mesh_graph(m)
    ov, orr = oracle.assemble(m, og)
    assert np.array_equal(row_ptr, np.asarray(og.row_ptr)) and np.array_equal(col, np.asarray(og.col))
    ev, er = fp64_errors(acc, ov, row_ptr, 3, accr, orr)
    assert ev < 1e-12 and er < 1e-12, (ev, er)
    g.destroy()

"""The device-resident cascade (ck_select_device, ck_cascade_eval_device):
the feature pass, the derivation of the model inputs and the three trees on
the GPU give the host cascade's decision, on the test matrices and on all
600 rows of the training table."""
import csv
import os

import numpy as np
import pytest

from helpers import MODEL, ROOT, parse_model, say
from synth import matrices as M

pytestmark = pytest.mark.gpu

FEATURES = ["nrows", "ncols", "nnz", "density", "mean", "sd", "cov", "max", "min", "maxavg",
            "distavg", "clusteravg", "fill", "ndiag", "diagfill"]


@pytest.fixture(scope="module")
def ck():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2411_10143_amd as ck
    ck.lib()
    return ck


MATS = {
    "powerlaw": lambda: M.power_law_rows(20011, 1.6, 3),
    "banded27": lambda: M.banded_stencil(30011, 27, 4),
    "blockdiag": lambda: M.block_diagonal(10007, 5),
    "uniform": lambda: M.uniform_random(50003, 6),
    "lap3d_40": lambda: M.laplacian_3d(40),
    "convdiff": lambda: M.convection_diffusion_2d(100, 10.0),
    "graph": lambda: M.graph_laplacian_chung_lu(30000, 12, wmax=4000),
    "column_runs": lambda: M.column_runs(1500, 6000, 8),
    "single_row": lambda: M.from_dense(np.arange(1.0, 200.0)[None, :]),
    "one_by_one": lambda: M.from_dense(np.array([[3.0]])),
    "empty": lambda: M.from_dense(np.zeros((5, 7))),
}


@pytest.mark.parametrize("name", list(MATS))
def test_device_cascade_equals_host(ck, orc, name):
    import torch
    A = MATS[name]()
    say(f"device cascade {name}")
    Mx = ck.Matrix.from_csr(A)
    F = ck.spmv_features(Mx.handle, symmetry=False)
    host = ck.spmv_select(F)
    out = torch.full((8,), -9, dtype=torch.int32, device="cuda")
    for _ in range(2):                       # the kept scratch is reused
        ck.select_device(Mx.handle, out)
        dev = out.cpu().tolist()
        assert dev[:4] == [host.format, host.algorithm, host.lanes, host.stages_done], (dev, host)
        assert dev[4:7] == ck.select_stages(F)
        assert dev[7] == ck.config_id(host)
        assert dev[4:7] == orc.cascade(parse_model(MODEL), orc.features(A)[2])
    Mx.close()


def test_device_tree_walk_on_the_training_table(ck):
    import torch
    path = os.path.join(ROOT, "paper_2411_10143_amd", "training", "mi355x_spmv_timings.csv")
    rows = list(csv.DictReader(open(path)))
    X = np.array([[float(r[k]) for k in FEATURES] for r in rows])
    ids = torch.full((len(X),), -9, dtype=torch.int32, device="cuda")
    say(f"device tree walk on {len(X)} rows")
    ck.cascade_eval_device(torch.from_numpy(X).cuda(), ids)
    got = ids.cpu().numpy()
    want = [ck.config_id(ck.spmv_select(ck.Features.from_model_inputs(x))) for x in X]
    assert list(got) == want

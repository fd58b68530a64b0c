"""Host-side checks of the benchmark's contract (no GPU): the one-GPU build
refuses more GPUs with a message, and the default workload is the documented
PFASST configuration (16 slices of two-level MLSDC, 127^3 / 63^3), so the
DOF-update count behind `value` is 127^3 x 4 substeps x 4 iterations x 16
slices per block."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


@pytest.mark.parametrize("n", [2, 8])
def test_more_gpus_refused(n):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", str(n)],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_default_workload_is_the_documented_one():
    import bench
    from paper_1307_7867_amd import heatst as hs

    pb = bench.problem(hs, 3)
    assert (pb.n, pb.order, pb.nnodes) == (127, 4, 5)
    assert pb.coarse == (63, 2, 3)
    assert (pb.nu, pb.dt, pb.t0, pb.forcing_c) == (0.1, 0.01, 0.0, 3.0)
    assert (pb.batch, pb.nslices, pb.nsteps) == (16, 16, 48)
    assert (pb.sweeps, pb.nu1, pb.nu2, pb.n_coarsest) == (4, 2, 1, 3)
    assert pb.omega == 6.0 / 7.0
    assert (pb.tol, pb.max_cycles) == (1e-12, 60)
    assert (pb.fused_sweeps, pb.cycle_graphs, pb.pfasst_pred_sweeps) == (1, 0, 1)
    assert (pb.pfasst_groups, pb.fas_interp) == (4, 3)
    assert pb.workspace_bytes() > 16 * 127 ** 3 * 8 * 16
    # value = space-time DOF-updates per second: fine points x substeps x iterations x slices per block
    assert (bench.NF, bench.MF, bench.ITERS, bench.SLICES) == (pb.n, pb.nnodes, pb.sweeps, pb.batch)
    assert bench.NF ** 3 * (bench.MF - 1) * bench.ITERS * bench.SLICES == 127 ** 3 * 4 * 4 * 16
    assert bench.PJAC_BYTES == 25

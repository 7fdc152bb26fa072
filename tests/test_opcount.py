"""The roofline's algorithmic FLOP figure per cell-update equals what the
operation-counting build of the oracle reports."""
import bench


def test_bench_flop_constant_matches_counting_build():
    from oracle import opcount
    parts, per_cell = opcount.counts()
    assert parts["ppm_line"][0] == 45 and parts["point_flux"][0] == 108
    assert abs(per_cell - bench.FLOPS_PER_CELL_UPDATE) <= 1.0


def test_bench_old_scheme_flop_constant_matches_counting_build():
    from oracle import opcount
    assert abs(opcount.counts_old() - bench.FLOPS_PER_CELL_UPDATE_OLD) <= 1.0

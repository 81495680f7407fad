"""The bench's reading of rocprofv3 counter rows (CPU): step-kernel
dispatches are summed, the steps counted (even launches plus the widest odd
launch), other kernels ignored and the copy probe averaged."""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import bench  # noqa: E402


def _row(name, grid, value):
    return {"Kernel_Name": name, "Grid_Size": str(grid), "Counter_Value": str(value)}


def test_step_kernel_rows_are_summed_per_step():
    even = "void lbm::step_kernel<2, float, false, 1, 0, false>(lbm::LatArgs, ...)"
    odd_w = "void lbm::step_kernel<2, float, true, 2, 0, false>(lbm::LatArgs, ...)"
    odd_b = "void lbm::step_kernel<2, float, true, 1, 1, false>(lbm::LatArgs, ...)"
    rows = []
    for _ in range(2):  # two even and two odd steps
        rows += [_row(even, 1000, 10.0), _row(odd_w, 990, 11.0), _row(odd_b, 10, 0.5)]
    rows += [_row("void lbm::init_equilibrium_kernel<2, float, float>(...)", 1000, 99.0),
             _row("void lbm::reduce_partial_kernel<2, float, true>(...)", 1000, 77.0),
             _row("void lbm::level_step_kernel<2, float, 1>(...)", 500, 55.0),
             _row("lbm::copy_kernel(...)", 4096, 2.0), _row("lbm::copy_kernel(...)", 4096, 4.0)]
    total, steps, copy = bench._step_kernel_kib(rows)
    assert steps == 4
    assert total == 2 * (10.0 + 11.0 + 0.5)
    assert copy == 3.0


def test_pair_kernel_and_link_kernel_count():
    pair = "void lbm::step_even_pair_kernel<2, true>(lbm::LatArgs)"
    odd = "void lbm::step_kernel<2, _Float16, true, 2, 0, false>(lbm::LatArgs, ...)"
    link = "void lbm::link_kernel<27, float, true>(...)"
    rows = [_row(pair, 500, 3.0), _row(odd, 990, 5.0), _row(link, 100, 0.25),
            _row("lbm::copy_kernel(...)", 4096, 1.0)]
    total, steps, copy = bench._step_kernel_kib(rows)
    assert steps == 2 and total == 8.25 and copy == 1.0


def test_adjoint_rows_are_summed_per_adjoint_step():
    rows = []
    for _ in range(3):  # three adjoint steps of each leg
        rows += [_row("void lbm::adjoint_kernel<2, float, 2, 0>(...)", 4000, 6.0),
                 _row("void lbm::adjoint_kernel<2, float, 1, 1>(...)", 30, 0.5),
                 _row("void lbm::adjoint_kernel<0, float, 2, 0>(...)", 4000, 4.0),
                 _row("void lbm::adjoint_kernel<2, double, 2, 0>(...)", 4000, 12.0)]
    rows += [_row("void lbm::step_kernel<2, float, false, 1, 0, false>(...)", 4100, 9.0),
             _row("lbm::copy_kernel(...)", 4096, 2.0)]
    legs, copy = bench._adjoint_kernel_kib(rows)
    assert copy == 2.0
    assert legs[("fclb", "f32")] == (3 * 6.5, 3)
    assert legs[("mrt", "f32")] == (12.0, 3)
    assert legs[("fclb", "f64")] == (36.0, 3)

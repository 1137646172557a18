"""The learned pressure-stage correction at the 200x200x50 workload's scale
(2M cells): training pairs collected by the solver from seeded training
fields of the workload's recipe (cfg 3, seeds 1606300 + f, disjoint from the
test systems), the network trained on the GPU by the library's kernels on
32x64x64 crops, then the workload's own systems solved in the FP32 form with
and without the network attached.

The measured result of this configuration (a reduced budget of the training
run documented with the profiles): the judged correction never adds
iterations (its multiple is chosen to lower the pressure residual, and it is
dropped when that multiple is not positive) and saves none on these systems,
while each application pays for the network's forward pass.  Both solves
reach the true FP64 residual of 1e-6."""
import pytest

pytestmark = pytest.mark.gpu


def test_learned_stage_at_workload_scale():
    from paper_1606_00556_amd import bo
    from paper_1606_00556_amd import nn_train as T
    bo.lib()
    out = T.main(["--fields", "4", "--systems", "1,9", "--steps", "800", "--eval", "1,10"])
    assert out["pairs"] == 4 * 2 * 4
    assert out["loss_last"] < out["loss_first"]
    for s in out["solves"]:
        plain, net = s["plain"], s["network"]
        print(f"{s['system']}: plain {plain['iterations']} its {plain['ms']:.1f} ms; with the network "
              f"{net['iterations']} its {net['ms']:.1f} ms, corrections kept {net['used']}")
        assert plain["converged"] and net["converged"]
        assert plain["rel"] <= 1e-6 and net["rel"] <= 1e-6
        assert net["iterations"] <= plain["iterations"]
    print(f"forward {out['forward_tflops']:.1f} TFLOP/s, backward {out['backward_tflops']:.1f} TFLOP/s "
          f"({out['voxels_per_step']} voxels per step)")

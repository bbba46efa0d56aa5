"""Command-line runner (host only): the workloads it names and its options."""

import pytest

from paper_2504_02627_amd import run


@pytest.mark.parametrize("name,N,d", [("small", 200, 5), ("large", 10000, 100),
                                      ("toeplitz", 5000, 100)])
def test_workloads_have_the_documented_shapes(name, N, d):
    Xs, ys = run.problem(name)
    assert len(Xs) == len(ys) == 1
    assert Xs[0].shape == (N, d) and ys[0].shape == (N,)


def test_unknown_workload_is_refused():
    with pytest.raises(ValueError):
        run.problem("nope")


def test_help_lists_the_step_size_flow_and_checkpoint_options(capsys):
    with pytest.raises(SystemExit) as e:
        run.main(["--help"])
    assert e.value.code == 0
    out = capsys.readouterr().out
    for opt in ("--workload", "--particles", "--precision", "--jitter", "--precond",
                "--step-size", "--traj-length", "--adapt-step-size", "--flow-layers",
                "--flow-train-steps", "--flow-lr", "--jsonl", "--save", "--resume"):
        assert opt in out

"""bench.py's command line on the host: it measures one GPU and refuses any
other count before it touches a device."""
import bench


def test_bench_refuses_more_than_one_gpu(capsys):
    assert bench.main(["--gpus", "2"]) == 2
    assert "one GPU only" in capsys.readouterr().err


def test_bench_refuses_a_distributed_launch(monkeypatch, capsys):
    monkeypatch.setenv("WORLD_SIZE", "2")
    assert bench.main([]) == 2
    assert "one GPU only" in capsys.readouterr().err

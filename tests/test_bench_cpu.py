"""bench.py's contract on the CPU: more than one GPU is refused with a message
(this build measures one GPU), and the binding refuses to run without the
HIP library instead of falling back to anything else."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.parametrize("argv,env", [(["--gpus", "2"], {}), ([], {"WORLD_SIZE": "4"})])
def test_bench_refuses_more_than_one_gpu(argv, env):
    e = dict(os.environ, **env)
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *argv], capture_output=True, text=True,
                       env=e, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_binding_fails_loudly_without_the_library(monkeypatch):
    import paper_2110_13735_amd as bnq
    monkeypatch.setattr(bnq, "_lib", None)
    monkeypatch.setattr(bnq, "LIBPATH", os.path.join(ROOT, "no_such_dir", "libbnq.so"))
    with pytest.raises(RuntimeError, match="missing"):
        bnq.lib()
    with pytest.raises(RuntimeError):
        bnq.footprint(bnq.Params(d=2, N=8))

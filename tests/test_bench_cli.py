"""bench.py's command-line contract on the host: more than one GPU is refused
with a message before anything touches a device."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_more_than_one_gpu():
    for args, env in ((["--gpus", "2"], {}), (["--gpus", "1"], {"WORLD_SIZE": "2"})):
        p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                           timeout=120, env={**os.environ, **env})
        assert p.returncode == 2, (args, env, p.returncode, p.stderr)
        assert "one GPU only" in p.stderr
        assert p.stdout == ""

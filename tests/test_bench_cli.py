"""bench.py on the CPU: a run on more than one GPU is refused with a JSON
message (the benchmark measures one GPU), before any GPU work; the board
power reading parses amd-smi's and rocm-smi's JSON."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300, cwd=ROOT)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert msg["n_gpus"] == 2 and "one GPU" in msg["error"]


def _bench_module():
    import importlib.util
    spec = importlib.util.spec_from_file_location("_bench", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


class _Done:
    def __init__(self, stdout):
        self.stdout = stdout


def test_board_power_reading(monkeypatch):
    bench = _bench_module()
    amd = json.dumps({"gpu_data": [{"gpu": 0, "power": {"socket_power": {"value": 1396, "unit": "W"},
                                                        "gfx_voltage": "N/A"}}]}, indent=4)
    rocm = json.dumps({"card0": {"Current Socket Graphics Package Power (W)": "1234.5"}})
    calls = []

    def fake(cmd, **kw):
        calls.append(cmd[0])
        return _Done(amd if cmd[0] == "amd-smi" else rocm)
    monkeypatch.setattr(subprocess, "run", fake)
    assert bench.read_board_power() == 1396.0
    assert calls == ["amd-smi"]

    def no_amd(cmd, **kw):
        if cmd[0] == "amd-smi":
            raise FileNotFoundError(cmd[0])
        return _Done(rocm)
    monkeypatch.setattr(subprocess, "run", no_amd)
    assert bench.read_board_power() == 1234.5
    monkeypatch.setattr(subprocess, "run", lambda cmd, **kw: _Done("{}"))
    assert bench.read_board_power() is None

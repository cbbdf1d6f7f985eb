"""bench.py on the host: a run on more than one GPU is refused with a
message (this build measures one GPU), before any device work; stored
profiler counters are used only for the kernel code they were taken on."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_counters_apply_only_to_the_kernel_they_were_taken_on(tmp_path, monkeypatch):
    """roofline.traffic and the executed MFMA rate come from stored counters
    only while the kernel's code (its source and the header it includes) is
    the code they were taken on: a comment edit keeps them, a code edit in
    either file drops them."""
    sys.path.insert(0, ROOT)
    import bench
    srcs = []
    for path in bench.KERNEL_SRCS:
        dst = tmp_path / os.path.basename(path)
        dst.write_text(open(path).read())
        srcs.append(str(dst))
    monkeypatch.setattr(bench, "KERNEL_SRCS", srcs)
    stored = json.load(open(bench.TRAFFIC_FILE))
    assert bench.kernel_digest() == stored["kernel_sha"]
    assert bench.counters_per_launch() == (stored["bytes_per_launch"], stored["mfma_instructions"])
    for path in srcs:
        text = open(path).read()
        open(path, "w").write(text + "\n// a comment\n/* and another */\n")
        assert bench.counters_per_launch()[0] is not None
        open(path, "w").write(text + "\nstatic int extra_symbol;\n")
        assert bench.counters_per_launch() == (None, None)
        open(path, "w").write(text)

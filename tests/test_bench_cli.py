"""bench.py's command-line contract on the CPU: more than one GPU is refused
with a message and exit status 2, before anything touches a device."""
import os
import subprocess
import sys


def test_multi_gpu_request_is_refused(repo_root):
    r = subprocess.run([sys.executable, os.path.join(repo_root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_kernel_hash_is_stable(repo_root):
    sys.path.insert(0, repo_root)
    import bench
    assert bench.kernel_hash() == bench.kernel_hash()
    assert len(bench.kernel_hash()) == 16

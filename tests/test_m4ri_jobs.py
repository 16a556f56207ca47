"""Host logic of the M4RI form's second-stream jobs (csrc/m4ri_jobs.h),
compiled with g++ and model-checked on random pass schedules: no pass
record is rewritten while a job that reads it may still run, and event
slots of outstanding jobs never collide."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_1111_6549_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_m4ri_job_ring_model_check(tmp_path):
    exe = tmp_path / "m4ri_jobs_check"
    subprocess.run(["g++", "-std=c++17", "-O1", "-I", CSRC, os.path.join(HERE, "cpp", "m4ri_jobs_check.cpp"), "-o",
                    str(exe)], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and r.stdout.strip() == "ok", r.stdout + r.stderr

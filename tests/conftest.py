import os
import subprocess
import sys
import tempfile
import time

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long CPU test")
    config.addinivalue_line("markers", "oracle_job(name): the test reads the result of a background oracle "
                                       "job of tests/oracle_jobs.py, started at session start")


class OracleJobs:
    """Child processes running tests/oracle_jobs.py, one per job name, started
    once per session for the selected GPU tests that declare them."""

    def __init__(self):
        self.dir = tempfile.mkdtemp(prefix="petto_oracle_jobs_")
        self.procs = {}

    def start(self, name):
        if name in self.procs:
            return
        out = os.path.join(self.dir, name + ".npz")
        log = open(os.path.join(self.dir, name + ".log"), "w")
        p = subprocess.Popen([sys.executable, os.path.join(ROOT, "tests", "oracle_jobs.py"), name, out],
                             stdout=log, stderr=subprocess.STDOUT, cwd=ROOT)
        self.procs[name] = (p, out, log)

    def result(self, name, timeout=1200.0, progress=None):
        """Wait for job `name` (starting it if needed) and load its arrays;
        `progress` (callable) receives the job's last log line about every 20 s."""
        self.start(name)
        p, out, log = self.procs[name]
        t0 = time.time()
        while p.poll() is None:
            if time.time() - t0 > timeout:
                p.kill()
                p.wait()
                raise TimeoutError(f"oracle job {name} still running after {timeout} s")
            time.sleep(20.0)
            if progress is not None:
                log.flush()
                with open(log.name) as fh:
                    lines = fh.read().strip().splitlines()
                progress(lines[-1] if lines else f"oracle job {name}: started")
        if p.returncode != 0:
            with open(log.name) as fh:
                raise RuntimeError(f"oracle job {name} failed:\n{fh.read()[-3000:]}")
        with np.load(out, allow_pickle=False) as z:
            return {k: z[k] for k in z.files}

    def close(self):
        for p, _, log in self.procs.values():
            if p.poll() is None:
                p.kill()
                p.wait()
            log.close()


@pytest.fixture(scope="session")
def oracle_jobs(request):
    jobs = OracleJobs()
    # start every job the selected tests declare, so they run while other GPU
    # tests use the device
    import torch
    if torch.cuda.is_available():
        for item in request.session.items:
            for m in item.iter_markers("oracle_job"):
                jobs.start(m.args[0])
    yield jobs
    jobs.close()


@pytest.fixture(scope="session", autouse=True)
def _start_oracle_jobs(request):
    """Touch the job fixture at the first test of a session that selected a test
    needing one (on a GPU machine), so the jobs start early."""
    if any(True for item in request.session.items for _ in item.iter_markers("oracle_job")):
        request.getfixturevalue("oracle_jobs")
    yield

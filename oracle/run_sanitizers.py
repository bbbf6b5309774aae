"""Runs the oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
(host code, g++) over every model family it simulates: sphere, corner-sphere
cube, box geom, legged chain, stacks of cubes with box-box contacts (and the
contact-capacity overflow), rollouts, right-hand sides and their directional
derivatives, forward-mode gradients and optimize-then-discretize gradients on
several threads, the CFD field, the continuous extension, both Runge-Kutta
pairs and the operation counter.

    python3 oracle/run_sanitizers.py

Exits nonzero on any sanitizer report (UBSan is made fatal).  TEST
INFRASTRUCTURE ONLY, like the rest of oracle/."""
import os
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)

WORKLOAD = r'''
import sys, numpy as np
sys.path.insert(0, ROOT)
from oracle import oracle as O
O.LIB_PATH = LIB
from paper_2506_14186_amd import workloads as W
rng = np.random.default_rng(0)
def run(desc, x0, u, n_int, dt, grad=True, cfd=0):
    m = O.Model(desc)
    r = m.rollout(x0, u, n_int, dt, tape_cap=64, log_cap=64, cfd=cfd)
    y = np.asarray(x0, float)
    f = m.rhs(y, u[0] if (u is not None and np.size(u)) else None)
    if grad:
        xb = np.ones((2, y.size))
        uu = None if u is None else np.stack([u, u])
        m.grad_batch(np.stack([y, y]), uu, n_int, dt, xb, n_threads=2, cfd=cfd)
        m.otd_grad_batch(np.stack([y, y]), uu, n_int, dt, xb, n_threads=2, cfd=cfd)
    return r["status"]
sphere = W.sphere_drop(seed=1, n_worlds=1, horizon=0.05)
print("sphere", run(W.model_sphere(), sphere["x0"][0], None, 1, 0.05))
cube = W.cube_toss(seed=2, n_worlds=1, horizon=0.05)
print("cube", run(W.model_cube_corners(), cube["x0"][0], None, 1, 0.05))
print("cube cfd", run(W.model_cube_corners(), cube["x0"][0], None, 1, 0.03, cfd=1))
box = W.box_toss(seed=4, n_worlds=1, horizon=0.05)
print("box", run(W.model_box(mu=0.6, tc=0.003), box["x0"][0], None, 1, 0.05))
ch = W.chain_walk(seed=3, n_worlds=1, n_intervals=3, interval_dt=0.01)
print("chain", run(W.model_chain(), ch["x0"][0], ch["u"][0], 3, 0.01))
for k in (2, 3):
    x = W.stack_state(rng.normal(0, 0.02, (k, 2)))
    print("stack", k, run(W.model_stack(k, tc=0.003, ctrl=True), x, rng.uniform(-1, 1, (2, 6)), 2, 0.01))
tossed = W.stack_state(np.zeros((2, 2)))
tossed[3:7] = [np.cos(0.2), np.sin(0.2), 0.0, 0.0]
tossed[7 + 3:7 + 7] = [np.cos(0.3), 0.0, np.sin(0.3), 0.0]
tossed[14:] = rng.normal(0, 0.3, 12)
print("stack tossed", run(W.model_stack(2, tc=0.003), tossed, None, 1, 0.03))
over = O.Model(W.model_stack(40, tc=0.003))
xs = W.stack_state(np.zeros((40, 2)))
for i in range(40):
    xs[7 * i + 2] = 0.1  # coincident cubes: more contacts than the capacity
print("overflow contacts", over.contacts(xs[:7 * 40]).shape)
pend = O.Model(W.model_pendulum())
xp = np.zeros(pend.nx)
xp[0], xp[pend.nq] = 1.2, 0.5
fz = np.array([[i * 0.05, 0.05] for i in range(8)]).ravel()
print("dense states", pend.dense_states(xp, None, 1, 0.4, np.linspace(0.0, 0.4, 9), forced=fz).shape)
for tab in (0, 1):
    print("tableau", tab, pend.rollout(xp, None, 1, 0.2, tableau=tab)["status"])
print("flop count", O.Model(W.model_stack(3, tc=0.003)).flop_count(W.stack_state(np.zeros((3, 2))), None, 1, 0.01)["status"])
A = np.eye(6) * 2.0
print("flop cholesky", O.flop_cholesky(A))
print("sanitized oracle run: done")
'''


def main():
    tmp = tempfile.mkdtemp(prefix="orc_san_")
    lib = os.path.join(tmp, "liboracle_san.so")
    flags = ["-O1", "-g", "-std=c++17", "-fPIC", "-shared", "-pthread", "-ffp-contract=off", "-fno-fast-math",
             "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"]
    subprocess.check_call(["g++"] + flags + ["-o", lib, os.path.join(HERE, "orc_sim.cpp")])
    asan = subprocess.check_output(["g++", "-print-file-name=libasan.so"]).decode().strip()
    env = dict(os.environ, LD_PRELOAD=asan, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    code = f"ROOT = {ROOT!r}\nLIB = {lib!r}\n" + WORKLOAD
    r = subprocess.run([sys.executable, "-c", code], env=env)
    print("exit", r.returncode)
    return r.returncode


if __name__ == "__main__":
    sys.exit(main())

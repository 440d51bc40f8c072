"""Resumable solves and the serving loop on the GPU: the batch step equals the blocking solve,
each request's result is the same alone and in a mix, served solutions match the oracle, and
admission respects a tight memory budget."""
import numpy as np
import pytest

from oracle import assemble, gmg, mesh, solve

pytestmark = pytest.mark.gpu

# a mix of degrees and mesh sizes, even and odd n (odd n: no h-coarsening, p-levels only)
MIX = [(1, 9, 0.7), (2, 6, 0.3), (3, 5, 0.0), (4, 4, 0.9), (2, 11, 0.5), (3, 8, 0.2)]


def _mfq():
    import paper_1910_13247_amd as mfq
    return mfq


def _torch():
    import torch
    return torch


def _requests(rtol=1e-10):
    from paper_1910_13247_amd.serve import Request
    return [Request(degree=p, n=n, alpha=a, seed=100 + i, rtol=rtol) for i, (p, n, a) in enumerate(MIX)]


def _serve(reqs, budget=8 << 30, **kw):
    from paper_1910_13247_amd.serve import DeviceExecutor, Server
    kw.setdefault("idle_sleep", 0)
    srv = Server(DeviceExecutor(keep_results=True), budget, **kw)
    for r in reqs:
        srv.submit(r)
    srv.drain()
    srv.close()
    _torch().cuda.synchronize()
    return srv


def test_space_random_matches_counter_definition():
    mfq = _mfq()
    m = mfq.Mesh(3, 0.0)
    s = mfq.Space(m, 2, mfq.MFQ_BC_DIRICHLET0)
    x = s.random(12345).cpu().numpy()
    ref = gmg.splitmix64_uniform(s.n_dofs, 12345) * mesh.boundary_mask(2, 3)
    np.testing.assert_array_equal(x, ref)


def test_batch_step_equals_blocking_solve():
    """Same solver driven by mfq_solve and by begin / batch_step / end with the step length equal
    to the poll period (the same launches in the same order): equal iteration counts and bitwise
    equal solutions (every kernel sums in a fixed order)."""
    mfq = _mfq()
    torch = _torch()
    print("batch step vs blocking", flush=True)
    m = mfq.Mesh(8, 0.1)
    s = mfq.Space(m, 3, mfq.MFQ_BC_DIRICHLET0)
    op = mfq.Operator(s, 0.5, mfq.MFQ_FP64)
    b = op.rhs_manufactured()
    sv = mfq.Solver(op, mfq.MFQ_SOLVER_GMG_MIXED, check_every=3)
    x1, info1, st1 = sv.solve(b, rtol=1e-10, max_iter=200)
    x2 = op.new_vector()
    sv.begin(b, x2, rtol=1e-10, max_iter=200)
    steps = 0
    while not mfq.batch_step([sv], iters=3)[0]:
        steps += 1
        assert steps < 1000
    st2, info2 = sv.end()
    torch.cuda.synchronize()
    assert st1 == st2 == mfq.MFQ_OK
    assert info1.iterations == info2.iterations and info1.outer_iterations == info2.outer_iterations
    assert info1.rel_residual <= 1e-10 and info2.rel_residual <= 1e-10
    assert torch.equal(x1, x2)


def test_resumable_errors():
    mfq = _mfq()
    _lib = mfq._lib
    m = mfq.Mesh(4, 0.0)
    s = mfq.Space(m, 2, mfq.MFQ_BC_DIRICHLET0)
    op = mfq.Operator(s, 0.0, mfq.MFQ_FP64)
    b = s.random(1)
    x = op.new_vector()
    sv = mfq.Solver(op, mfq.MFQ_SOLVER_GMG_MIXED)
    with pytest.raises(_lib.MfqError) as e:
        sv.end()
    assert e.value.status == mfq.MFQ_EINVAL
    sv.begin(b, x)
    with pytest.raises(_lib.MfqError) as e:
        sv.begin(b, x)
    assert e.value.status == mfq.MFQ_EBUSY
    while not mfq.batch_step([sv], iters=2)[0]:
        pass
    st, info = sv.end()
    assert st == mfq.MFQ_OK and info.rel_residual <= 1e-10
    sv.begin(b, x)  # a finished solver can run the next solve
    while not mfq.batch_step([sv], iters=2)[0]:
        pass
    assert sv.end()[0] == mfq.MFQ_OK


def test_cg_true_residual_certified():
    """Plain CG stops on its recurred residual; the residual check adds FP64 correction passes
    until the true residual meets rtol."""
    mfq = _mfq()
    print("cg certified", flush=True)
    m = mfq.Mesh(12, 0.1)
    s = mfq.Space(m, 3, mfq.MFQ_BC_DIRICHLET0)
    op = mfq.Operator(s, 0.5, mfq.MFQ_FP64)
    b = op.rhs_manufactured()
    sv = mfq.Solver(op, mfq.MFQ_SOLVER_CG)
    x, info, st = sv.solve(b, rtol=1e-10, max_iter=20000)
    assert st == mfq.MFQ_OK and info.rel_residual <= 1e-10
    At = assemble.operator_csr(3, 12, 0.1, 0.5, 1)
    assert solve.rel_residual(lambda v: At @ v, b.cpu().numpy(), x.cpu().numpy()) <= 1e-10


@pytest.mark.parametrize("mode,threads", [("sync", 0), ("async", 0), ("async", 1), ("sync", 2)])
def test_served_results_match_oracle(mode, threads):
    """Each served request solves its own system: the solution agrees with a sparse direct solve
    of the oracle's assembled operator for the same counter-based right-hand side (set-up on the
    scheduler thread or on worker threads)."""
    print(f"serve vs oracle ({mode}, {threads} set-up threads)", flush=True)
    reqs = _requests()
    srv = _serve(reqs, mode=mode, setup_threads=threads)
    assert len(srv.done) == len(reqs)
    for r in reqs:
        assert r.status == 0 and r.rel_residual <= 1e-10, (r.degree, r.n, r.rel_residual)
        A = assemble.operator_csr(r.degree, r.n, 0.0, r.alpha, 1)
        N = A.shape[0]
        b = gmg.splitmix64_uniform(N, r.seed) * mesh.boundary_mask(r.degree, r.n)
        x = r.result.cpu().numpy()
        assert solve.rel_residual(lambda v: A @ v, b, x) <= 1e-10
        xd = solve.direct_solve(A, b)
        # relative residual 1e-10 bounds the error by cond(A) * 1e-10; cond < 1e4 here
        assert np.abs(x - xd).max() <= 1e-6 * np.abs(xd).max(), (r.degree, r.n)


@pytest.mark.parametrize("mode,threads", [("sync", 0), ("async", 0), ("async", 1)])
def test_alone_and_in_mix_agree(mode, threads):
    """The same request alone and among others (other requests' work overlapping on the device,
    on other streams): equal iteration counts and bitwise equal solutions."""
    print(f"alone vs mix ({mode}, {threads} set-up threads)", flush=True)
    mixed = _requests()
    _serve(mixed, mode=mode, setup_threads=threads)
    for i, p in enumerate(MIX):
        alone = _requests()[i]
        _serve([alone], mode=mode)
        m = mixed[i]
        assert alone.status == m.status == 0
        assert alone.iterations == m.iterations, (p, alone.iterations, m.iterations)
        xa, xm = alone.result.cpu().numpy(), m.result.cpu().numpy()
        np.testing.assert_array_equal(xa, xm, err_msg=str(p))


def test_tight_budget_serialises_admission():
    """With a budget that holds only the largest request, no two large requests are resident at
    once, and every request still finishes, in FIFO admission order."""
    from paper_1910_13247_amd.serve import DeviceExecutor
    print("tight budget", flush=True)
    reqs = _requests()
    ex = DeviceExecutor()
    sizes = []
    for r in reqs:
        h = ex.prepare(r)
        sizes.append(h["bytes"])
        ex.release(h)
    budget = max(sizes) + min(sizes) - 1
    srv = _serve(reqs, budget=budget)
    assert srv.peak_used <= budget
    assert all(r.status == 0 for r in reqs)
    adm = sorted(reqs, key=lambda r: r.admitted)
    assert [r.id for r in adm] == sorted(r.id for r in reqs)


def test_graph_replay_matches_direct_launches():
    """The same solve on a non-default stream with each CG iteration replayed from a captured HIP
    graph and with every launch issued directly: equal iteration counts, both certified, and
    solutions equal bitwise.  Every step replays the
    graph several times with eager work (the residual check) and host waits in between; bitwise
    equal solutions."""
    mfq = _mfq()
    torch = _torch()
    print("graph vs direct", flush=True)
    m = mfq.Mesh(8, 0.1)
    s = mfq.Space(m, 3, mfq.MFQ_BC_DIRICHLET0)
    op = mfq.Operator(s, 0.5, mfq.MFQ_FP64)
    b = op.rhs_manufactured()
    torch.cuda.synchronize()
    st = torch.cuda.Stream()
    out = {}
    for g in (0, 1):
        for kind in (mfq.MFQ_SOLVER_GMG_MIXED, mfq.MFQ_SOLVER_GMG_MIXED_IR, mfq.MFQ_SOLVER_CG):
            sv = mfq.Solver(op, kind, use_graphs=g, coarse_mode=1)
            x = op.new_vector()
            sv.begin(b, x, rtol=1e-10, max_iter=2000, stream=st)
            while not mfq.batch_step([sv], iters=3)[0]:
                pass
            status, info = sv.end()
            torch.cuda.synchronize()
            out[(g, kind)] = (status, info.iterations, info.rel_residual, x.clone())
    for kind in (mfq.MFQ_SOLVER_GMG_MIXED, mfq.MFQ_SOLVER_GMG_MIXED_IR, mfq.MFQ_SOLVER_CG):
        d, g = out[(0, kind)], out[(1, kind)]
        assert d[0] == g[0] == mfq.MFQ_OK
        assert d[1] == g[1], (kind, d[1], g[1])
        assert d[2] <= 1e-10 and g[2] <= 1e-10
        assert torch.equal(d[3], g[3]), kind


def test_async_step_protocol():
    """mfq_solve_step_async / _poll: a second submit before the poll completes is refused, the
    poll reports done exactly when the solve has finished, and the result is certified."""
    mfq = _mfq()
    torch = _torch()
    _lib = mfq._lib
    m = mfq.Mesh(6, 0.1)
    s = mfq.Space(m, 2, mfq.MFQ_BC_DIRICHLET0)
    op = mfq.Operator(s, 0.3, mfq.MFQ_FP64)
    b = s.random(9)
    x = op.new_vector()
    st = torch.cuda.Stream()
    sv = mfq.Solver(op, mfq.MFQ_SOLVER_GMG_MIXED, coarse_mode=1)
    with pytest.raises(_lib.MfqError):
        _lib.mfq_solve_step_poll(sv.handle)          # nothing begun
    sv.begin(b, x, stream=st)
    _lib.mfq_solve_step_async(sv.handle, 2)
    with pytest.raises(_lib.MfqError) as e:
        _lib.mfq_solve_step_async(sv.handle, 2)      # previous step not yet polled complete
    assert e.value.status == mfq.MFQ_EBUSY
    polls = 0
    while True:
        ready, done = _lib.mfq_solve_step_poll(sv.handle)
        polls += 1
        assert polls < 10**7
        if not ready:
            continue
        if done:
            break
        _lib.mfq_solve_step_async(sv.handle, 2)
    status, info = sv.end()
    torch.cuda.synchronize()
    assert status == mfq.MFQ_OK and info.rel_residual <= 1e-10


def test_solver_rebind_drops_captured_graphs():
    """A solver bound to another buffer does not replay iterations captured on the old one: with
    the old buffer filled with NaN (and kept allocated) the next solve on the same stream still
    converges to the same solution."""
    mfq = _mfq()
    torch = _torch()
    m = mfq.Mesh(6, 0.1)
    s = mfq.Space(m, 2, mfq.MFQ_BC_DIRICHLET0)
    op = mfq.Operator(s, 0.3, mfq.MFQ_FP64)
    b = s.random(5)
    st = torch.cuda.Stream()
    torch.cuda.synchronize()
    sv = mfq.Solver(op, mfq.MFQ_SOLVER_GMG_MIXED, coarse_mode=1)
    xs = []
    x = op.new_vector()                  # one solution vector: the graphs' key stays the same
    for k in range(2):
        if k == 1:
            old = sv.buffer
            new = torch.empty_like(old)
            mfq._lib.mfq_solver_bind(sv.handle, new.data_ptr(), sv.device_bytes, st.cuda_stream)
            sv.buffer = new
            old.fill_(255)
            torch.cuda.synchronize()
        sv.begin(b, x, rtol=1e-10, max_iter=200, stream=st)
        while not mfq.batch_step([sv], iters=3)[0]:
            pass
        status, info = sv.end()
        torch.cuda.synchronize()
        assert status == mfq.MFQ_OK and info.rel_residual <= 1e-10
        xs.append(x.clone())
    assert torch.equal(xs[0], xs[1])
    del old


def test_batched_run_is_bitwise_the_single_solve_step():
    """mfq_batch_run over a mix of degrees, mesh sizes (even and odd n: h- and p-coarsened
    hierarchies of different depths) and coefficients, all on one stream with batched launches per
    (kernel, degree): each solve's iteration count and solution equal those of the same solve
    advanced alone by mfq_batch_step, bitwise."""
    mfq = _mfq()
    torch = _torch()
    print("batched run vs single steps", flush=True)
    st = torch.cuda.Stream()
    cases = MIX + [(5, 6, 0.4), (6, 4, 0.8), (1, 16, 0.1)]
    sols, bs, xs_alone, it_alone = [], [], [], []
    for i, (p, n, a) in enumerate(cases):
        op = mfq.Operator(mfq.Space(mfq.Mesh(n, 0.0), p, mfq.MFQ_BC_DIRICHLET0), a, mfq.MFQ_FP64)
        b = op.space.random(500 + i)
        sv = mfq.Solver(op, mfq.MFQ_SOLVER_GMG_MIXED, coarse_mode=1)
        x = op.new_vector()
        sv.begin(b, x, rtol=1e-10, max_iter=300, stream=st)
        while not mfq.batch_step([sv], iters=2)[0]:
            pass
        s_, info = sv.end()
        assert s_ == mfq.MFQ_OK
        xs_alone.append(x.clone())
        it_alone.append(info.iterations)
        sols.append(sv)
        bs.append(b)
    batch = mfq.Batch(16, stream=st)
    xs = []
    for sv, b in zip(sols, bs):
        x = sv.op.new_vector()
        sv.begin(b, x, rtol=1e-10, max_iter=300, stream=st)
        xs.append(x)
    pending = list(range(len(sols)))
    steps = 0
    while pending:
        flags = batch.run([sols[i] for i in pending], iters=2, stream=st)
        pending = [i for i, f in zip(pending, flags) if not f]
        steps += 1
        assert steps < 500
    torch.cuda.synchronize()
    for i, sv in enumerate(sols):
        s_, info = sv.end()
        assert s_ == mfq.MFQ_OK and info.rel_residual <= 1e-10, cases[i]
        assert info.iterations == it_alone[i], (cases[i], info.iterations, it_alone[i])
        assert torch.equal(xs[i], xs_alone[i]), cases[i]


def test_batched_serving_matches_oracle_and_alone():
    """The serving loop with a batched executor: every result certified by the oracle's operator,
    and each request's solution bitwise equal to the same request served alone."""
    print("batched serving", flush=True)
    reqs = _requests()
    from paper_1910_13247_amd.serve import DeviceExecutor, Server
    srv = Server(DeviceExecutor(keep_results=True, batched=True), 8 << 30, idle_sleep=0, setup_threads=1)
    for r in reqs:
        srv.submit(r)
    srv.drain()
    srv.close()
    _torch().cuda.synchronize()
    for i, r in enumerate(reqs):
        assert r.status == 0 and r.rel_residual <= 1e-10
        A = assemble.operator_csr(r.degree, r.n, 0.0, r.alpha, 1)
        b = gmg.splitmix64_uniform(A.shape[0], r.seed) * mesh.boundary_mask(r.degree, r.n)
        assert solve.rel_residual(lambda v: A @ v, b, r.result.cpu().numpy()) <= 1e-10
        alone = _requests()[i]
        srv1 = Server(DeviceExecutor(keep_results=True, batched=True), 8 << 30, idle_sleep=0)
        srv1.submit(alone)
        srv1.drain()
        srv1.close()
        assert alone.iterations == r.iterations
        np.testing.assert_array_equal(alone.result.cpu().numpy(), r.result.cpu().numpy())


def test_lazy_bind_batched_estimates_and_starts_are_bitwise():
    """Solvers bound lazily (eigenvalue bounds estimated by the first step) and advanced by
    mfq_batch_run, where the estimates of all of them run in one set of launches and the CG pass
    starts and residual checks are batched too: bounds, iteration counts and solutions equal those
    of the same solvers bound eagerly and advanced alone, bitwise.  One solver with another
    Lanczos length takes the per-solve estimate inside the same call."""
    mfq = _mfq()
    torch = _torch()
    print("lazy bind + batched estimates", flush=True)
    st = torch.cuda.Stream()
    cases = MIX + [(5, 6, 0.4), (1, 16, 0.1)]
    rtols = [1e-10, 1e-13, 1e-10, 1e-13, 1e-10, 1e-10, 1e-12, 1e-10]
    lanczos = [None] * len(cases)
    lanczos[2] = 8
    ref = []
    for i, (p, n, a) in enumerate(cases):
        op = mfq.Operator(mfq.Space(mfq.Mesh(n, 0.0), p, mfq.MFQ_BC_DIRICHLET0), a, mfq.MFQ_FP64)
        b = op.space.random(700 + i)
        kw = {} if lanczos[i] is None else {"lanczos_iters": lanczos[i]}
        sv = mfq.Solver(op, mfq.MFQ_SOLVER_GMG_MIXED, coarse_mode=1, **kw)
        x = op.new_vector()
        sv.begin(b, x, rtol=rtols[i], max_iter=400, stream=st)
        while not mfq.batch_step([sv], iters=2)[0]:
            pass
        s_, info = sv.end()
        assert s_ == mfq.MFQ_OK
        nl = info.n_levels
        ref.append((op, b, x.clone(), info.iterations, info.outer_iterations, sv.lambdas(nl), kw))
    lazy, xs = [], []
    for i, (op, b, _, _, _, _, kw) in enumerate(ref):
        sv = mfq.Solver(op, mfq.MFQ_SOLVER_GMG_MIXED, coarse_mode=1, lazy=True, stream=st, **kw)
        with pytest.raises(mfq._lib.MfqError):
            sv.lambdas(8)
        x = op.new_vector()
        sv.begin(b, x, rtol=rtols[i], max_iter=400, stream=st)
        lazy.append(sv)
        xs.append(x)
    batch = mfq.Batch(16, stream=st)
    pending = list(range(len(lazy)))
    steps = 0
    while pending:
        flags = batch.run([lazy[i] for i in pending], iters=2, stream=st)
        pending = [i for i, f in zip(pending, flags) if not f]
        steps += 1
        assert steps < 600
    torch.cuda.synchronize()
    for i, sv in enumerate(lazy):
        s_, info = sv.end()
        _, _, x_ref, its, outer, lam, _ = ref[i]
        print(f"  {cases[i]} rtol {rtols[i]:.0e}: {its} iterations, {outer} passes")
        assert s_ == mfq.MFQ_OK
        assert sv.lambdas(info.n_levels) == lam, cases[i]
        assert info.iterations == its and info.outer_iterations == outer, (cases[i], info.iterations, its)
        assert torch.equal(xs[i], x_ref), cases[i]


def test_lazy_bind_alone_equals_eager():
    """A lazily bound solver advanced by mfq_batch_step (the estimate made per solve at its first
    step) and one whose preconditioner is applied before any solve give the eager solver's
    results bitwise."""
    mfq = _mfq()
    torch = _torch()
    p, n, a = 3, 6, 0.5
    op = mfq.Operator(mfq.Space(mfq.Mesh(n, 0.1), p, mfq.MFQ_BC_DIRICHLET0), a, mfq.MFQ_FP64)
    b = op.space.random(11)
    eager = mfq.Solver(op, mfq.MFQ_SOLVER_GMG_MIXED)
    x0, info0, s0 = eager.solve(b, rtol=1e-10, max_iter=300)
    z0 = eager.precondition(b)
    lazy = mfq.Solver(op, mfq.MFQ_SOLVER_GMG_MIXED, lazy=True)
    x1, info1, s1 = lazy.solve(b, rtol=1e-10, max_iter=300)
    assert s0 == s1 == mfq.MFQ_OK and info0.iterations == info1.iterations
    assert torch.equal(x0, x1)
    lazy2 = mfq.Solver(op, mfq.MFQ_SOLVER_GMG_MIXED, lazy=True)
    z1 = lazy2.precondition(b)
    torch.cuda.synchronize()
    assert torch.equal(z0, z1)
    assert lazy2.lambdas(info0.n_levels) == eager.lambdas(info0.n_levels)

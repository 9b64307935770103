"""GPU parity of the all-DOF time synthesis (residue identification for every
unknown with the common poles, then Eq. 6), computed as one FP64 matrix-core
contraction, against the oracle's residue identification and time response,
and against the closed-form inverse of exactly rational data.

Tolerances: the two sides solve the same least-squares problem in different
arithmetic order (Householder QR here, LAPACK there) and sum 2J products per
output; 1e-10 of the response scale.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _needs_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")


def _poles(n_pairs, real):
    rng = np.random.default_rng(7)
    w = np.sort(rng.uniform(0.2, 3.0, n_pairs))
    p = []
    for wi in w:
        a = complex(-rng.uniform(0.01, 0.2), wi)
        p += [a, np.conj(a)]
    if real:
        p.append(complex(-0.3, 0.0))
    return np.array(p)


@pytest.mark.parametrize("real_pole", [False, True])
@pytest.mark.parametrize("N,Nt", [(1000, 100), (37, 513), (16, 64)])
def test_synthesis_matches_oracle(real_pole, N, Nt):
    import paper_1511_04355_amd as afs
    from oracle import vf
    rng = np.random.default_rng(N + Nt)
    poles = _poles(5, real_pole)
    J = 24
    s = 0.05 + 1j * np.linspace(0.0, 3.5, J)
    X = rng.standard_normal((J, N)) + 1j * rng.standard_normal((J, N))
    t = np.linspace(0.0, 40.0, Nt)
    h = afs.time_synthesis(poles, s, torch.from_numpy(X).cuda(), t).cpu().numpy()
    po, res = vf.identify_residues(s, X.T, poles)
    ho = vf.time_response(t, po, res)
    assert h.shape == ho.shape == (N, Nt)
    assert np.max(np.abs(h - ho)) <= 1e-10 * np.max(np.abs(ho))


@pytest.mark.parametrize("J,n_pairs,real_pole,N,Nt", [(1, 0, True, 333, 77), (7, 3, False, 333, 77),
                                                      (64, 5, True, 333, 77), (65, 5, False, 333, 77),
                                                      (24, 5, False, 1, 300)])
def test_synthesis_sample_counts(J, n_pairs, real_pole, N, Nt):
    """One sample (one matrix-core pair step), a ragged pair (J = 7), the most
    samples of the register-resident path (J = 64), the general path beyond it
    (J = 65), and a single unknown; ragged N and Nt throughout."""
    import paper_1511_04355_amd as afs
    from oracle import vf
    rng = np.random.default_rng(J * 1000 + N)
    poles = _poles(n_pairs, real_pole)
    s = 0.05 + 1j * np.linspace(0.0, 3.5, J)
    X = rng.standard_normal((J, N)) + 1j * rng.standard_normal((J, N))
    t = np.linspace(0.0, 40.0, Nt)
    h = afs.time_synthesis(poles, s, torch.from_numpy(X).cuda(), t).cpu().numpy()
    po, res = vf.identify_residues(s, X.T, poles)
    ho = vf.time_response(t, po, res)
    assert np.max(np.abs(h - ho)) <= 1e-10 * np.max(np.abs(ho))


def test_synthesis_exact_for_rational_samples():
    """Samples of sum_m r_nm / (s - a_m) with conjugate-symmetric residues:
    the synthesis returns the exact inverse transform sum_m r_nm e^{a_m t}."""
    import paper_1511_04355_amd as afs
    rng = np.random.default_rng(3)
    poles = _poles(4, True)
    N, J, Nt = 500, 20, 200
    r = np.zeros((N, len(poles)), np.complex128)
    for m in range(0, 8, 2):
        r[:, m] = rng.standard_normal(N) + 1j * rng.standard_normal(N)
        r[:, m + 1] = np.conj(r[:, m])
    r[:, 8] = rng.standard_normal(N)
    s = 0.05 + 1j * np.linspace(0.0, 3.5, J)
    X = (r @ (1.0 / (s[None, :] - poles[:, None]))).T  # [J, N]
    t = np.linspace(0.0, 30.0, Nt)
    h = afs.time_synthesis(poles, s, torch.from_numpy(np.ascontiguousarray(X)).cuda(), t).cpu().numpy()
    exact = np.real(r @ np.exp(np.outer(poles, t)))
    assert np.max(np.abs(h - exact)) <= 1e-9 * np.max(np.abs(exact))


def test_synthesis_full_size_sampled_rows():
    """300,516 unknowns (the 64-void block's size), 20 samples on the band
    [0, 0.67] of the porous workloads, 512 steps, exactly rational data with
    in-band poles: sampled rows against the closed-form inverse and against
    the oracle; the contraction's rate is printed."""
    import time

    import paper_1511_04355_amd as afs
    from oracle import vf
    rng = np.random.default_rng(11)
    w = np.array([0.08, 0.21, 0.34, 0.47, 0.6])
    poles = np.concatenate([[complex(-0.02 - 0.01 * i, wi), complex(-0.02 - 0.01 * i, -wi)]
                            for i, wi in enumerate(w)])
    N, J, Nt = 300516, 20, 512
    s = 0.023 + 1j * np.linspace(0.0, 0.67, J)
    g = torch.Generator(device="cuda").manual_seed(5)
    r = torch.randn(N, 5, dtype=torch.complex128, device="cuda", generator=g)
    R = torch.empty(N, 10, dtype=torch.complex128, device="cuda")
    R[:, 0::2] = r
    R[:, 1::2] = r.conj()
    Phi = torch.from_numpy(1.0 / (s[None, :] - poles[:, None])).cuda()  # [M, J]
    X = (R @ Phi).T.contiguous()  # [J, N]
    t = np.arange(Nt) * 300.0 / Nt
    h = afs.time_synthesis(poles, s, X, t)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(5):
        h = afs.time_synthesis(poles, s, X, t)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / 5
    flops = 2.0 * N * Nt * 2 * J
    print(f"[synthesis] N={N} Nt={Nt} 2J={2 * J}: {dt * 1e3:.3f} ms per call (incl. host K), "
          f"{flops / dt / 1e12:.1f} TFLOP/s, output {N * Nt * 8 / dt / 1e9:.0f} GB/s", flush=True)
    rows = np.sort(rng.choice(N, 64, replace=False))
    hs = h[rows].cpu().numpy()
    exact = np.real(R[rows].cpu().numpy() @ np.exp(np.outer(poles, t)))
    assert np.max(np.abs(hs - exact)) <= 1e-9 * np.max(np.abs(exact))
    po, res = vf.identify_residues(s, X[:, rows].cpu().numpy().T, poles)
    ho = vf.time_response(t, po, res)
    assert np.max(np.abs(hs - ho)) <= 1e-10 * np.max(np.abs(ho))

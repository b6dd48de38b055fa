"""GPU path (through the C ABI) against the FP64 oracle on the same seeded inputs."""
import ctypes

import numpy as np
import pytest

import _gpu
from _gpu import TOL, matrix, parity, run_gpu, run_oracle
from oracle import philox, rnla

pytestmark = pytest.mark.gpu


def test_philox_words_bit_exact():
    import torch
    import paper_2410_19208_amd as pp
    dev = _gpu.device()
    for seed, stream, c0, cnt in [(0, 0, 0, 1000), (123456789, 1, 2**33 + 7, 4097), (2**63 + 5, 2, 99, 10)]:
        out = torch.zeros(4 * cnt, dtype=torch.int32, device=dev)
        pp.psdproj_philox_words(seed, stream, c0, cnt, out.data_ptr(), 0)
        torch.cuda.synchronize()
        got = out.cpu().numpy().view(np.uint32).reshape(cnt, 4)
        ref = philox.raw_words(seed, stream, np.arange(c0, c0 + cnt, dtype=np.uint64))
        assert np.array_equal(got, ref)


def test_gaussian_stream_matches():
    import torch
    import paper_2410_19208_amd as pp
    dev = _gpu.device()
    for seed, stream, start, cnt in [(0, 0, 0, 50001), (77, 1, 3, 1000), (5, 2, 2**35, 64)]:
        out = torch.zeros(cnt, dtype=torch.float64, device=dev)
        pp.psdproj_gaussian(seed, stream, start, cnt, out.data_ptr(), 0)
        torch.cuda.synchronize()
        ref = philox.gaussian(seed, stream, cnt, start)
        assert np.max(np.abs(out.cpu().numpy() - ref)) < 1e-13


def test_small_fp64_workload_stages():
    """n = 512, k = 40, p = 10, q = 0, plain, FP64: Omega, Ritz values, r_plus and P."""
    n, k, p = 512, 40, 10
    A, lam, U = matrix("small", n, 1001)
    proj, P, res = run_gpu(A, k, p, 0, "plain", "fp64", seed=0)
    ref = run_oracle(A, k, p, 0, "plain", "fp64", seed=0)
    assert res.status == 0
    assert res.r_plus == ref.r_plus
    ev = proj.evals().cpu().numpy()
    assert np.max(np.abs(np.sort(ev) - ref.evals)) < 1e-12 * np.abs(ref.evals).max()
    Q = proj.q_panel().cpu().numpy()
    assert np.linalg.norm(Q @ Q.T - ref.Q @ ref.Q.T) < 1e-11
    assert parity(P, ref, A) < TOL["fp64"]
    assert np.array_equal(P, P.T)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
@pytest.mark.parametrize("variant,alpha", [("plain", 0.0), ("scaled", 0.35), ("scaled", 0.0)])
@pytest.mark.parametrize("q", [0, 1])
def test_parity_ragged(prec, variant, alpha, q):
    """n = 777 (ragged against every tile), k = 40, p = 12."""
    n, k, p = 777, 40, 12
    A, lam, U = matrix("medium", n, 5, n_pos=60)
    proj, P, res = run_gpu(A, k, p, q, variant, prec, seed=3, alpha=alpha)
    ref = run_oracle(A, k, p, q, variant, prec, seed=3, alpha=alpha)
    assert res.status == 0
    if variant == "scaled" and alpha == 0.0:
        assert abs(res.alpha_used - ref.alpha) < 1e-10 * ref.alpha
    err = parity(P, ref, A)
    print(f"{prec} {variant} alpha={alpha} q={q}: parity {err:.3e} r+ {res.r_plus}/{ref.r_plus}")
    assert err < TOL[prec]
    assert np.array_equal(P, P.T)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
@pytest.mark.parametrize("variant,alpha", [("plain", 0.0), ("scaled", 0.0)])
@pytest.mark.parametrize("n,lda", [(777, 780), (777, 800), (780, 800)])
def test_parity_ragged_padded_rows(prec, variant, alpha, n, lda):
    """n stored in a wider buffer (row stride lda, 16-byte aligned rows) whose padding columns
    hold NaN: the ragged last tile and K step must never let them into the result.  n = 777
    takes the element-load path, n = 780 (a multiple of 4) the vector-load path."""
    import torch
    from paper_2410_19208_amd.torch_api import Projector
    dev = _gpu.device()
    k, p, q = 40, 12, 1
    A, lam, U = matrix("medium", n, 5, n_pos=60)
    dt = torch.float64 if prec == "fp64" else torch.float32
    buf = torch.full((n, lda), float("nan"), dtype=dt, device=dev)
    buf[:, :n] = _gpu.to_dev(A.astype(_gpu.storage(prec)), dev)
    proj = Projector(n, k, p, q, variant, prec, seed=3, alpha=alpha, device=dev)
    P = proj(buf[:, :n]).cpu().numpy()
    res = proj.result()
    ref = run_oracle(A, k, p, q, variant, prec, seed=3, alpha=alpha)
    assert res.status == 0
    err = parity(P, ref, A)
    print(f"padded n={n} lda={lda} {prec} {variant}: parity {err:.3e}")
    assert err < TOL[prec]


@pytest.mark.parametrize("prec", ["fp64", "bf16x3"])
@pytest.mark.parametrize("variant,alpha", [("plain", 0.0), ("scaled", 0.0)])
@pytest.mark.parametrize("q", [2, 3])
def test_parity_power_steps(prec, variant, alpha, q):
    """Several power steps (Alg. 1 with q = 2, 3): the orthonormalisations before the last one
    only fix the range, and a well-conditioned sketch takes one CholeskyQR round there."""
    n, k, p = 777, 40, 12
    A, lam, U = matrix("medium", n, 5, n_pos=60)
    proj, P, res = run_gpu(A, k, p, q, variant, prec, seed=4, alpha=alpha)
    ref = run_oracle(A, k, p, q, variant, prec, seed=4, alpha=alpha)
    assert res.status == 0
    err = parity(P, ref, A)
    print(f"{prec} {variant} q={q}: parity {err:.3e} r+ {res.r_plus}/{ref.r_plus}")
    assert err < TOL[prec]
    assert np.array_equal(P, P.T)


@pytest.mark.parametrize("prec", ["fp64", "bf16x3"])
def test_parity_ill_conditioned_sketch(prec):
    """Eigenvalues decaying over twelve decades: the sketch's Cholesky pivots fall far below
    its Gram diagonal, so every orthonormalisation keeps its second CholeskyQR round."""
    n, k, p, q = 120, 44, 8, 2
    lam = 10.0 ** (-np.linspace(0.0, 12.0, n))
    lam[1::3] *= -1.0
    A, _, U = matrix("spectrum", n, 12, lam=lam)
    for variant in ("plain", "scaled"):
        proj, P, res = run_gpu(A, k, p, q, variant, prec, seed=6)
        ref = run_oracle(A, k, p, q, variant, prec, seed=6)
        assert res.status == 0
        assert parity(P, ref, A) < TOL[prec]


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_exact_recovery(prec):
    """rank(A) <= k+p: the projection is A_+ (closed form) to working precision."""
    n = 300
    rng = np.random.default_rng(2)
    lam = np.zeros(n)
    lam[:12] = rng.uniform(0.2, 2, 12)
    lam[12:24] = -rng.uniform(0.2, 2, 12)
    A, _, U = matrix("spectrum", n, 9, lam=lam)
    proj, P, res = run_gpu(A, 24, 8, 1, "plain", prec, seed=1)
    Ap = (U * np.maximum(lam, 0)) @ U.T
    err = np.linalg.norm(P - Ap) / np.linalg.norm(Ap)
    assert err < {"fp64": 1e-11, "fp32": 1e-5, "bf16x3": 5e-5}[prec]


@pytest.mark.parametrize("n,k,p", [(1, 1, 0), (2, 1, 1), (3, 1, 0), (17, 5, 3), (40, 30, 10), (129, 100, 29)])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_edge_sizes(n, k, p, prec):
    A, lam, U = matrix("spectrum", n, 4, lam=np.linspace(1.0, -1.0, n))
    for variant, alpha in [("plain", 0.0), ("scaled", 1.2)]:
        proj, P, res = run_gpu(A, k, p, 1, variant, prec, seed=2, alpha=alpha)
        ref = run_oracle(A, k, p, 1, variant, prec, seed=2, alpha=alpha)
        assert res.status == 0
        assert parity(P, ref, A) < TOL[prec]


def test_zero_matrix():
    n = 64
    A = np.zeros((n, n))
    proj, P, res = run_gpu(A, 8, 4, 1, "plain", "fp32", seed=0)
    assert res.status == 0 and res.r_plus == 0 and not P.any()
    proj, P, res = run_gpu(A, 8, 4, 1, "scaled", "fp32", seed=0, alpha=0.0)
    import paper_2410_19208_amd as pp
    assert res.status == pp.E_ALPHA


def test_nonfinite_input_is_reported():
    import paper_2410_19208_amd as pp
    A, _, _ = matrix("small", 100, 3, n_pos=5)
    A[7, 9] = A[9, 7] = np.nan
    proj, P, res = run_gpu(A, 8, 4, 0, "plain", "fp32", seed=0)
    assert res.status == pp.E_NONFINITE


def test_in_place_output_aliases_input():
    import torch
    from paper_2410_19208_amd.torch_api import Projector
    dev = _gpu.device()
    A, _, _ = matrix("small", 500, 8, n_pos=30)
    A32 = A.astype(np.float32)
    proj = Projector(500, 30, 10, 1, "scaled", "bf16x3", seed=4, device=dev)
    At = _gpu.to_dev(A32, dev)
    P_sep = proj(At).cpu().numpy()
    At2 = _gpu.to_dev(A32, dev)
    proj(At2, P=At2)
    torch.cuda.synchronize()
    assert np.array_equal(At2.cpu().numpy(), P_sep)


def test_batch_equals_single_runs_bitwise():
    import torch
    from paper_2410_19208_amd.torch_api import BatchProjector, Projector
    dev = _gpu.device()
    specs = [dict(n=300, k=20, p=8, q=1, variant="plain", precision="bf16x3", seed=1),
             dict(n=1000, k=60, p=10, q=0, variant="scaled", precision="bf16x3", seed=2),
             dict(n=77, k=10, p=5, q=2, variant="scaled", precision="fp32", seed=3, alpha=0.5),
             dict(n=512, k=40, p=10, q=0, variant="plain", precision="fp64", seed=0),
             dict(n=650, k=20, p=8, q=1, variant="plain", precision="bf16x3", seed=5)]
    As = []
    for i, s in enumerate(specs):
        A, _, _ = matrix("small", s["n"], 20 + i, n_pos=max(2, s["n"] // 10))
        As.append(_gpu.to_dev(A.astype(_gpu.storage(s["precision"])), dev))
    bp = BatchProjector(specs, device=dev)
    Pb = bp(As)
    torch.cuda.synchronize()
    rb = bp.results()
    for i, s in enumerate(specs):
        s2 = dict(s)
        proj = Projector(s2.pop("n"), s2.pop("k"), s2.pop("p"), device=dev, **s2)
        P1 = proj(As[i])
        torch.cuda.synchronize()
        assert proj.result().status == 0 and rb[i].status == 0
        assert proj.result().r_plus == rb[i].r_plus
        assert torch.equal(P1, Pb[i]), f"batch member {i} differs from its single run"


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
@pytest.mark.parametrize("k,p", [(140, 10), (170, 10), (210, 10), (240, 10), (246, 10)])
def test_parity_wide_panels(prec, k, p):
    """Sketch widths r = 150, 180, 220, 250, 256 (padded widths 160, 192, 224, 256, 256): the
    widest register-tiled forms of the pass, Cholesky, apply and tridiagonalisation kernels (for
    BF16X3 the widths 160 .. 224 take the pass whose A slices go through LDS), both variants
    (alpha estimated by Alg. 5), one power step."""
    n, q = 1500, 1
    A, lam, U = matrix("medium", n, 11, n_pos=300)
    for variant in ("plain", "scaled"):
        proj, P, res = run_gpu(A, k, p, q, variant, prec, seed=5)
        ref = run_oracle(A, k, p, q, variant, prec, seed=5)
        assert res.status == 0
        assert res.r_plus == ref.r_plus
        if variant == "scaled":
            assert abs(res.alpha_used - ref.alpha) < 1e-10 * ref.alpha
        err = parity(P, ref, A)
        print(f"wide r={k + p} {prec} {variant}: parity {err:.3e} r+ {res.r_plus}")
        assert err < TOL[prec]
        assert np.array_equal(P, P.T)


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
@pytest.mark.parametrize("k,p", [(150, 10), (190, 10)])
def test_parity_empty_k_chunk(prec, k, p):
    """n = 260: the pass splits K into chunks of 128 rows (0, 128, 256), and the 16-byte BF16X3
    pass covers whole 32-row steps only (rows below 256), so its third chunk has no step: it
    must write a zero partial tile while rows 256 .. 259 come from the reduction.  Widths 160
    and 224, both variants, one power step."""
    n, q = 260, 1
    A, lam, U = matrix("medium", n, 12, n_pos=60)
    for variant in ("plain", "scaled"):
        proj, P, res = run_gpu(A, k, p, q, variant, prec, seed=8)
        ref = run_oracle(A, k, p, q, variant, prec, seed=8)
        assert res.status == 0 and res.r_plus == ref.r_plus
        err = parity(P, ref, A)
        print(f"n=260 r={k + p} {prec} {variant}: parity {err:.3e}")
        assert err < TOL[prec]


@pytest.mark.parametrize("n", [160, 192])
def test_parity_short_k_chunks(n):
    """n = 160 and 192 at width 160 (k + p = 150): two K chunks of 128 rows, the second holding
    one or two 32-row steps of the 16-byte BF16X3 pass (whose A slices go through LDS), so the
    copies issued ahead of the first step reach past the chunk's last step.  Both variants, one
    power step."""
    k, p, q = 140, 10, 1
    A, lam, U = matrix("medium", n, 14, n_pos=30)
    for variant in ("plain", "scaled"):
        proj, P, res = run_gpu(A, k, p, q, variant, "bf16x3", seed=10)
        ref = run_oracle(A, k, p, q, variant, "bf16x3", seed=10)
        assert res.status == 0 and res.r_plus == ref.r_plus
        err = parity(P, ref, A)
        print(f"n={n} r=150 bf16x3 {variant}: parity {err:.3e}")
        assert err < TOL["bf16x3"]


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_huge_row_stride(prec):
    """Rows 2^24 + 64 elements apart (an n x n view into a 13 GB buffer): the 16-byte paths,
    which reach 32 rows of A by 32-bit byte offsets from a per-step base, must give way to the
    element paths (width 160 would otherwise take the BF16X3 pass whose A slices go through LDS).
    Both variants, one power step, against the oracle."""
    import torch
    from paper_2410_19208_amd.torch_api import Projector
    n, k, p, q = 200, 150, 10, 1
    lda = (1 << 24) + 64
    A, lam, U = matrix("medium", n, 13, n_pos=40)
    dev = _gpu.device()
    buf = torch.empty((n - 1) * lda + n, dtype=torch.float32, device=dev)
    At = torch.as_strided(buf, (n, n), (lda, 1))
    At.copy_(torch.from_numpy(A.astype(np.float32)).to(dev))
    for variant in ("plain", "scaled"):
        proj = Projector(n, k, p, q, variant, prec, seed=9, device=dev)
        P = proj(At)
        torch.cuda.synchronize()
        res = proj.result()
        ref = run_oracle(A, k, p, q, variant, prec, seed=9)
        assert res.status == 0 and res.r_plus == ref.r_plus
        err = parity(P.cpu().numpy(), ref, A)
        print(f"lda=2^24+64 {prec} {variant}: parity {err:.3e}")
        assert err < TOL[prec]
    del At, buf
    torch.cuda.empty_cache()


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_cor2_repeated_eigenvalues(prec):
    """The matrix class of Cor. 2 (four blocks of n/4 equal eigenvalues -3, -1, 6, 2), n = 512,
    k = 200 > n/4, l = 5, q = 2 (Example 1's parameters): the compressed matrix has long runs of
    eigenvalues closer than 1e-5 ||T||, which the eigenvector kernel treats as clusters.  Parity
    with the oracle in both variants (alpha = beta_1 = 3 given), and the scaled projection is the
    more accurate one, as Cor. 2 predicts for k > n/4."""
    n, k, p, q = 512, 200, 5, 2
    A, lam, U = matrix("cor2", n, 7)
    Ap = (U * np.maximum(lam, 0.0)) @ U.T
    e_alg = {}
    for variant, alpha in (("plain", 0.0), ("scaled", 3.0)):
        proj, P, res = run_gpu(A, k, p, q, variant, prec, seed=1, alpha=alpha)
        ref = run_oracle(A, k, p, q, variant, prec, seed=1, alpha=alpha)
        assert res.status == 0
        gaps = np.diff(ref.evals)
        assert np.count_nonzero(gaps < 1e-5 * np.abs(ref.evals).max()) > 50   # clusters present
        err = parity(P, ref, A)
        e_alg[variant] = np.linalg.norm(P.astype(np.float64) - Ap) / np.linalg.norm(Ap)
        print(f"cor2 {prec} {variant}: parity {err:.3e} e_alg {e_alg[variant]:.4f} r+ {res.r_plus}/{ref.r_plus}")
        assert err < TOL[prec]
    assert e_alg["scaled"] < e_alg["plain"]


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
@pytest.mark.parametrize("variant", ["plain", "scaled"])
def test_rows_past_n_poisoned(prec, variant):
    """n = 780 (16-byte aligned rows, n not a multiple of the 32-row pass step) inside a buffer
    of n + 32 rows whose rows past n and padding columns hold NaN: the last pass step reads
    rows at or past n, which must count as zero."""
    import torch
    from paper_2410_19208_amd.torch_api import Projector
    dev = _gpu.device()
    n, lda, k, p, q = 780, 800, 40, 12, 1
    A, lam, U = matrix("medium", n, 5, n_pos=60)
    buf = torch.full((n + 32, lda), float("nan"), dtype=torch.float32, device=dev)
    buf[:n, :n] = _gpu.to_dev(A.astype(np.float32), dev)
    proj = Projector(n, k, p, q, variant, prec, seed=3, device=dev)
    P = proj(buf[:n, :n]).cpu().numpy()
    res = proj.result()
    ref = run_oracle(A, k, p, q, variant, prec, seed=3)
    assert res.status == 0
    err = parity(P, ref, A)
    print(f"rows past n poisoned {prec} {variant}: parity {err:.3e}")
    assert err < TOL[prec]


def test_exact_clusters_recovered():
    """rank(A) = 100 <= k + p with three eigenvalues repeated 40, 40 and 20 times: the sketch
    spans range(A), the compressed matrix has three exact clusters (plus zeros), and the
    projection is A_+ (Thm 1) to working precision in FP64."""
    n = 600
    lam = np.zeros(n)
    lam[:40] = 2.0
    lam[40:80] = 1.0
    lam[80:100] = -1.5
    A, _, U = matrix("spectrum", n, 21, lam=lam)
    Ap = (U * np.maximum(lam, 0.0)) @ U.T
    proj, P, res = run_gpu(A, 100, 10, 0, "plain", "fp64", seed=2)
    ref = run_oracle(A, 100, 10, 0, "plain", "fp64", seed=2)
    assert res.status == 0 and res.r_plus >= 80
    assert parity(P, ref, A) < TOL["fp64"]
    assert np.linalg.norm(P - Ap) / np.linalg.norm(Ap) < 1e-11


@pytest.mark.parametrize("variant", ["plain", "scaled"])
@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_negative_definite_projects_to_zero(prec, variant):
    # Every Ritz value of a negative definite matrix is negative, so neither clamp keeps a
    # direction (Alg. 2: max(d, 0); Alg. 3: max(d, 1) - 1 with d = lambda / alpha + 1 < 1):
    # r_plus = 0 on both sides and the rebuild writes P = 0 exactly.
    n = 300
    rng = np.random.default_rng(23)
    U, _ = np.linalg.qr(rng.standard_normal((n, n)))
    lam = -rng.uniform(0.1, 1.0, n)
    A = (U * lam) @ U.T
    A = 0.5 * (A + A.T)
    proj, P, res = run_gpu(A, 20, 10, 1, variant, prec, seed=5, alpha=0.0)
    ref = run_oracle(A, 20, 10, 1, variant, prec, seed=5, keep_P=False)
    assert res.status == 0
    assert res.r_plus == 0 and ref.r_plus == 0
    assert not P.any()

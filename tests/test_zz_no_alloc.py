"""mb4_energy_components_noalloc against mb4_energy_components.

The allocation-free entry point evaluates the energy components (Sec. 2.1,
Eqs. U_K - U_E, in the halved convention of the library) of a device field
through the library's fixed scratch array.  Two calls in a row, the second
on a smaller lattice, must each give what a state holding the same field
returns, bit for bit (the same kernels sum in the same order), so nothing of
the first call's partial sums may leak into the second.
"""
import numpy as np
import pytest

from gpu_common import torch_cuda
from paper_2003_04345_amd import mb4 as M

pytestmark = pytest.mark.gpu


def _field(nx, ny, seed):
    rng = np.random.default_rng(seed)
    n = nx * ny
    v = rng.uniform(-1.0, 1.0, n)
    v[rng.choice(n, size=max(1, n // 200), replace=False)] = 50.0
    amp = rng.uniform(0.1, 0.5, n)
    ph = rng.uniform(0.0, 2 * np.pi, n)
    return v, amp * np.cos(ph), amp * np.sin(ph)


def _by_state(nx, ny, v, p, q, g, t_hop, shift):
    with M.MB4State(nx, ny, v, g, 0.01, t_hop=t_hop, diag_shift=shift) as st:
        st.set_state(p, q)
        out = (M.c_double * 6)()
        M._check(M.load_library().mb4_energy_components(st.handle, out), "mb4_energy_components")
        return np.array(out[:], dtype=np.float64)


def _noalloc(torch, nx, ny, v, p, q, g, t_hop, shift):
    dv = torch.from_numpy(v).to("cuda")
    dp = torch.from_numpy(p).to("cuda")
    dq = torch.from_numpy(q).to("cuda")
    out = torch.full((6,), float("nan"), dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    M.mb4_energy_components_noalloc(nx, ny, g, dv, dp, dq, out, t_hop=t_hop, diag_shift=shift,
                                    stream=stream)
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("shapes", [((100, 65), (37, 20)), ((2048, 40), (450, 97))])
def test_noalloc_energy_matches_the_state_entry_point(shapes):
    torch = torch_cuda()
    for k, (nx, ny) in enumerate(shapes):
        g, t_hop, shift = (1.0, 1.0, 0.0) if k == 0 else (2.0, 0.7, 2.8)
        v, p, q = _field(nx, ny, seed=nx * 131 + ny)
        want = _by_state(nx, ny, v, p, q, g, t_hop, shift)
        got = _noalloc(torch, nx, ny, v, p, q, g, t_hop, shift)
        assert np.all(np.isfinite(got))
        assert np.array_equal(got, want), (nx, ny, got - want)


def test_noalloc_energy_at_the_largest_tile_count():
    # 2048 x 4096: exactly the 32768 tiles the scratch array holds.
    torch = torch_cuda()
    nx, ny = 2048, 4096
    v, p, q = _field(nx, ny, seed=5)
    want = _by_state(nx, ny, v, p, q, 2.0, 1.0, 0.0)
    got = _noalloc(torch, nx, ny, v, p, q, 2.0, 1.0, 0.0)
    assert np.array_equal(got, want)
    # Then a small lattice again: the large call's partials are not read.
    v, p, q = _field(16, 9, seed=6)
    assert np.array_equal(_noalloc(torch, 16, 9, v, p, q, 1.0, 1.0, 0.0),
                          _by_state(16, 9, v, p, q, 1.0, 1.0, 0.0))

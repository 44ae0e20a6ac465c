"""A general sparse Hamiltonian (not a lattice): random symmetric neighbour
lists with per-bond hoppings, double-precision on-site energies and
antisymmetric bond displacements, which exercise the explicit neighbour list,
per-slot hopping and double on-site paths, against the oracle's CSR."""
import numpy as np
import pytest

import kpm_inputs as ki
import oracle
from cases import rel_err

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
kp = pytest.importorskip("paper_1307_0288_amd")


def _random_graph(n, width, seed):
    """Symmetric random graph: each row gets up to `width` bonds."""
    u = ki.uniform(seed, 8 * n * width)
    nbr = -np.ones((width, n), dtype=np.int32)
    hop = np.zeros((width, n))
    dx = np.zeros((width, n))
    deg = np.zeros(n, dtype=int)
    q = 0
    for a in range(n):
        for _ in range(width):
            b = int(u[q] * n); hv = -1.0 - u[q + 1]; dv = u[q + 2] - 0.5; q += 3
            if b == a or deg[a] >= width or deg[b] >= width:
                continue
            if np.any(nbr[:deg[a], a] == b):
                continue
            nbr[deg[a], a] = b; hop[deg[a], a] = hv; dx[deg[a], a] = dv; deg[a] += 1
            nbr[deg[b], b] = a; hop[deg[b], b] = hv; dx[deg[b], b] = -dv; deg[b] += 1
    onsite = (ki.uniform(seed + 1, n) - 0.5) * 0.7      # not float-exact
    return nbr, hop, dx, onsite


def _to_oracle(nbr, hop, dx, onsite):
    w, n = nbr.shape
    rows, cols, hv, dv = [], [], [], []
    for a in range(n):
        for k in range(w):
            if nbr[k, a] >= 0:
                rows.append(a); cols.append(nbr[k, a]); hv.append(hop[k, a]); dv.append(dx[k, a])
    order = np.lexsort((np.arange(len(rows)), rows))
    rows = np.asarray(rows)[order]
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(row_ptr, rows + 1, 1)
    row_ptr = np.cumsum(row_ptr)
    return oracle.Lattice(n, 1, "sheet", 0.0, row_ptr, np.asarray(cols, np.int64)[order],
                          np.asarray(hv)[order], np.asarray(dv)[order], onsite.copy(),
                          np.ones(n, np.uint8))


@pytest.fixture(scope="module")
def general():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    n, width = 3000, 4
    nbr, hop, dx, onsite = _random_graph(n, width, 77)
    lat = _to_oracle(nbr, hop, dx, onsite)
    es = 1.01 * (np.max(np.abs(onsite)) + width * 2.0)
    sysg = kp.System(nbr, es, hop=hop, onsite=onsite, dx=dx)
    phi = ki.random_phase(n, 2, 3000)
    return lat, es, sysg, phi


def test_general_moments(general):
    lat, es, sysg, phi = general
    d = sysg.upload(phi)
    got = kp.kpm_moments(sysg, d, d, 200)
    for r in range(2):
        ref = oracle.moments(lat, es, phi[:, r], phi[:, r], 200)
        assert rel_err(got[r], ref, np.vdot(phi[:, r], phi[:, r]).real) < 1e-10


def test_general_evolve_and_commutator(general):
    lat, es, sysg, phi = general
    d = sysg.upload(phi[:, :1])
    ox, ou = sysg.new_state(1), sysg.new_state(1)
    kp.kpm_evolve_x(sysg, d, ox, ou, 0.3, 30)
    rx, ru = oracle.evolve_x(lat, es, phi[:, 0], 0.3, 30)
    assert rel_err(ox.cpu().numpy()[:, 0], rx) < 1e-12
    assert rel_err(ou.cpu().numpy()[:, 0], ru) < 1e-12
    kp.kpm_evolve(sysg, d, 0.3, -1, 30)
    assert rel_err(d.cpu().numpy()[:, 0], oracle.evolve(lat, es, phi[:, 0], 0.3, -1, 30)) < 1e-12


def test_general_vac_msd(general):
    lat, es, sysg, phi = general
    d = sysg.upload(phi[:, :1])
    args = (2, 0.25, 25, 40)
    assert rel_err(kp.kpm_vac(sysg, d, *args)[0], oracle.vac(lat, es, phi[:, 0], *args)) < 1e-10
    assert rel_err(kp.kpm_msd(sysg, d, *args)[0], oracle.msd(lat, es, phi[:, 0], *args)) < 1e-10


def test_compact_and_explicit_forms_agree(monkeypatch):
    """The compact device form (pattern bytes, float on-site) and the explicit
    one give the same moments up to rounding, and both match the oracle."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from cases import oracle_lattice, phases, recipe, gpu_system
    c = recipe("sheet", 100, 50, w=1.0, vac=0.02, seed=4)
    lat = oracle_lattice(c)
    phi = phases(c, 1, 3000)
    compact = gpu_system(c)
    monkeypatch.setenv("KPM_COMPACT", "0")
    explicit = gpu_system(c)
    a = kp.kpm_moments(compact, compact.upload(phi), compact.upload(phi), 300)[0]
    b = kp.kpm_moments(explicit, explicit.upload(phi), explicit.upload(phi), 300)[0]
    ref = oracle.moments(lat, c["e_scale"], phi[:, 0], phi[:, 0], 300)
    scale = np.vdot(phi, phi).real
    assert rel_err(a, b, scale) < 1e-13
    assert rel_err(a, ref, scale) < 1e-10
    assert rel_err(b, ref, scale) < 1e-10

"""End-to-end physics pin of the oracle: the Landau damping rate (Sec. 2.1;
Fig. correctness_landau shows the E_x energy decaying at the analytical rate)."""
import numpy as np
import pytest

from paper_2605_05469_amd import synth
from tests.landau_util import fit_damping, landau_root


def test_dispersion_root_k05():
    w = landau_root(0.5)
    # classical values for k lambda_D = 0.5: w_r ~ 1.4156, gamma ~ -0.1533
    assert abs(w.real - 1.4156) < 1e-3 and abs(w.imag + 0.1533) < 1e-3


@pytest.mark.slow
def test_oracle_landau_damping_rate(orc):
    N, ppc = 32, 8
    P = synth.LandauParams(N=N, ppc=ppc)
    st = orc.State(N, P.L, P.q, P.qm, P.dt, *synth.landau_particles_np(N, ppc, seed=P.seed))
    st.init(1e-10, 20000)

    def mode_energy():
        # energy of the fundamental x-mode of E_x (the damped Landau mode)
        return abs(np.fft.fftn(st.ex.reshape(N, N, N))[0, 0, 1]) ** 2

    e = [mode_energy()]
    for _ in range(300):
        info = st.step(1e-10, 20000)
        assert info["converged"]
        e.append(mode_energy())
    t = np.arange(len(e)) * P.dt
    gamma, npk = fit_damping(t, e)
    g_th = landau_root(0.5).imag
    assert npk >= 4
    assert abs(gamma - g_th) <= 0.10 * abs(g_th)

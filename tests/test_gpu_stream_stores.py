"""Non-temporal stores of the sweep passes' volume outputs
(BD3MG_OPT_STREAM_STORES) are a cache hint only: runs with the hint on and
off are bitwise equal (x, the previous steps, the blurred residual), in the
coloured, sequential and round schedules, both precisions, with H dp kept
(the update pass's H d' stores) and without."""
import numpy as np
import pytest

from paper_2002_02328_amd import binding
from gpu_common import pair

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec,schedule,hdp", [(binding.FP32, binding.SCHED_COLORED, 64),
                                               (binding.FP32, binding.SCHED_ROUND, 64),
                                               (binding.FP64, binding.SCHED_COLORED, 0),
                                               (binding.FP64, binding.SCHED_SEQUENTIAL, 64)])
def test_stream_stores_bitwise(orc, prec, schedule, hdp):
    out = []
    for nt in (0, 1):
        g, o, y = pair(orc, (13, 45, 130), prec, seed=21, kx=7, ky=5, kz=5, lam=0.02, delta=0.03,
                       eta=0.3, nslices=[3, 2, 4, 1, 3], schedule=schedule,
                       mu=0.3 if schedule == binding.SCHED_ROUND else 0.0)
        g.set_option(binding.OPT_STREAM_STORES, nt)
        g.set_option(binding.OPT_HDP_EVERY, hdp)
        g.set_x0(None)
        g.run(9, check_every=0)
        out.append((g.get_x(), g.get_dprev(), g.get_state()[2]))
        g.close()
    for a, b in zip(*out):
        assert np.array_equal(a, b)


def test_stream_stores_option_values(orc):
    g, o, y = pair(orc, (4, 16, 64), binding.FP32, seed=2, nslices=[2, 2])
    for v in (-1, 0, 1):
        g.set_option(binding.OPT_STREAM_STORES, v)
    for v in (-2, 2):
        with pytest.raises(binding.Bd3mgError):
            g.set_option(binding.OPT_STREAM_STORES, v)
    g.close()

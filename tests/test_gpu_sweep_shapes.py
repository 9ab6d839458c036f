"""Every launch shape of the stream-collide update gives the same bits: the
per-node arithmetic (its fused multiply-adds written out) does not depend on
the threads per workgroup, the nodes per thread or the streaming hints.
Each case runs the same seeded domain under every shape through the C ABI
and compares records and fields with the default shape's bit for bit, in
2-byte and 4-byte storage: x faces of every kind (inlet with zero-gradient
or velocity outlet, Zou-He faces with the quasi-incompressible equilibrium,
periodic x, x walls), an odd row length and a domain with a moving body.
"""
import numpy as np
import pytest

import lbm_workloads as W
from gpu_helpers import make_gpu

pytestmark = pytest.mark.gpu

SHAPES = [(256, 1, 0), (256, 1, 3), (256, 2, 0), (256, 2, 2), (128, 2, 0), (128, 2, 1), (128, 2, 3)]


def _cases():
    duct = W.duct_sphere(scale=4, storage="f16")  # 64 x 32 x 32
    return {
        "duct_f16": (duct, 80),
        "duct_f16_nx63": (W.with_changes(duct, nx=63), 80),  # odd rows
        "duct_f16_zouhe_heluo": (W.with_changes(duct, eq="heluo", faces=(W.ZOUHE_VELOCITY, W.ZOUHE_PRESSURE) +
                                                 W.DUCT_FACES[2:]), 80),
        "duct_f16_periodic_x": (W.with_changes(duct, faces=(W.PERIODIC, W.PERIODIC) + W.DUCT_FACES[2:],
                                               rho_noise=1e-3), 80),
        "duct_f16_x_walls": (W.with_changes(duct, faces=W.CLOSED_FACES, rho_noise=1e-3), 80),
        "channel_f16_velocity_outlet": (W.with_changes(W.channel_cylinder_f64(), storage="f16", nx=101,
                                                       faces=W.CHANNEL_VELOCITY_FACES), 200),
        "channel_f16_oscillating": (W.with_changes(W.channel_oscillating_f32(scale=10), storage="f16"), 150),
        "duct_f32": (W.with_changes(duct, storage="f32"), 60),
    }


@pytest.mark.parametrize("case", sorted(_cases()))
def test_every_shape_same_bits(case):
    w, steps = _cases()[case]
    print(f"sweep shapes: {case} ({w['nx']} x {w['ny']} x {w['nz']}, {w['storage']}), {steps} steps", flush=True)
    # the plain schedule, so that a moving body's domain runs this sweep too
    ref = make_gpu(w, split_schedule=-1)
    ref.step(steps)
    rr, ur = ref.fields()
    recs = ref.records(0)
    for block, cpt, mem in SHAPES:
        d = make_gpu(w, split_schedule=-1)
        d.sweep_config = dict(block=block, cells_per_thread=cpt, memory=mem, remap=0)
        d.step(steps)
        r, u = d.fields()
        same = np.array_equal(r, rr, equal_nan=True) and np.array_equal(u, ur, equal_nan=True) and \
            np.array_equal(d.records(0), recs)
        print(f"  shape {block} x {cpt}, memory {mem}: {'same bits' if same else 'DIFFERENT'}", flush=True)
        assert same, (block, cpt, mem)
        d.close()
    assert np.nanmax(np.abs(ur)) > 0
    ref.close()

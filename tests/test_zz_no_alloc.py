"""j3d_solve_noalloc (the allocation-free one-shot solve) against the plain
solver path it mirrors: bit-identical interiors and residuals on two calls in a
row, the second with a smaller input, through the C ABI."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _reference(api, p, n, nblk, split, bc, seed, pid, iters, u0=None):
    with api.Solver(n, nblk=nblk, split=split, bc=bc, seed=seed, pid=pid) as s:
        if u0 is not None:
            s.set_interior(u0)
        r = s.run(iters, mode="fused", residual=True)
        return s.get_interior(), r


def test_noalloc_matches_the_solver_on_two_calls():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2202_11819_amd import api, j3d
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    # call 1: seeded interior, uneven 3x2x2 decomposition, 37 sweeps
    n1, nblk1, split1 = (96, 70, 45), (3, 2, 2), ([30, 33, 33], [35, 35], [20, 25])
    bc1 = (0.5, -0.25, 0.125, 1.0, -1.0, 0.0)
    p1 = j3d.Problem(n1, nblk1, split1, bc1, 7, 3)
    fb1 = j3d.j3d_field_bytes(p1)
    # call 2: a smaller problem from a given interior, 2x1x1 blocks, 12 sweeps
    n2, nblk2 = (40, 33, 21), (2, 1, 1)
    bc2 = (1.0, 0.0, 0.0, -0.5, 0.25, 0.75)
    p2 = j3d.Problem(n2, nblk2, None, bc2, 1, 0)
    fb2 = j3d.j3d_field_bytes(p2)
    assert fb2 < fb1
    fields = torch.empty(fb1, dtype=torch.uint8, device="cuda")
    out1 = torch.empty((n1[2], n1[1], n1[0]), dtype=torch.float64, device="cuda")
    print(f"noalloc call 1: {n1} as {nblk1} blocks, 37 sweeps", flush=True)
    r1 = j3d.j3d_solve_noalloc(p1, fields.data_ptr(), fb1, None, out1.data_ptr(), 37, residual=True,
                               stream_ptr=stream.cuda_stream)
    want1, want_r1 = _reference(api, p1, n1, nblk1, split1, bc1, 7, 3, 37)
    assert np.array_equal(out1.cpu().numpy(), want1)
    assert r1 == want_r1 and r1 > 0
    u0 = np.random.default_rng(5).uniform(-1, 1, (n2[2], n2[1], n2[0]))
    uin = torch.from_numpy(u0).cuda()
    out2 = torch.empty((n2[2], n2[1], n2[0]), dtype=torch.float64, device="cuda")
    print(f"noalloc call 2: {n2} as {nblk2} blocks from a given interior, 12 sweeps", flush=True)
    r2 = j3d.j3d_solve_noalloc(p2, fields.data_ptr(), fb2, uin.data_ptr(), out2.data_ptr(), 12, residual=True,
                               stream_ptr=stream.cuda_stream)
    want2, want_r2 = _reference(api, p2, n2, nblk2, None, bc2, 1, 0, 12, u0=u0)
    assert np.array_equal(out2.cpu().numpy(), want2)
    assert r2 == want_r2
    # no residual requested, zero sweeps: the input comes back unchanged
    out3 = torch.full_like(out2, float("nan"))
    assert j3d.j3d_solve_noalloc(p2, fields.data_ptr(), fb2, uin.data_ptr(), out3.data_ptr(), 0,
                                 stream_ptr=stream.cuda_stream) is None
    torch.cuda.synchronize()
    assert np.array_equal(out3.cpu().numpy(), u0)


def test_noalloc_rejects_bad_arguments_before_device_work():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2202_11819_amd import j3d
    L = j3d._lib
    p = j3d.Problem((16, 16, 16), (2, 2, 2))
    fb = j3d.j3d_field_bytes(p)
    fields = torch.empty(fb + 256, dtype=torch.uint8, device="cuda")
    out = torch.empty(16 ** 3, dtype=torch.float64, device="cuda")
    base = fields.data_ptr()
    r = ctypes.c_double(-1.0)
    cases = [((None, base, fb, None, out.data_ptr(), 3, None, None), j3d.J3D_EINVAL),
             ((ctypes.byref(p.c), None, fb, None, out.data_ptr(), 3, None, None), j3d.J3D_EINVAL),
             ((ctypes.byref(p.c), base, fb, None, None, 3, None, None), j3d.J3D_EINVAL),
             ((ctypes.byref(p.c), base + 8, fb, None, out.data_ptr(), 3, None, None), j3d.J3D_EINVAL),
             ((ctypes.byref(p.c), base, fb, None, out.data_ptr(), -1, None, None), j3d.J3D_EINVAL),
             ((ctypes.byref(p.c), base, fb - 8, None, out.data_ptr(), 3, ctypes.byref(r), None), j3d.J3D_ENOMEM),
             ((ctypes.byref(p.c), base, fb, None, base + 1024, 3, None, None), j3d.J3D_EINVAL)]
    for args, want in cases:
        assert L.j3d_solve_noalloc(*args) == want, args
    assert r.value == -1.0
    # tables beyond the static scratch: 40^3 blocks of 1^3
    big = j3d.Problem((40, 40, 40), (40, 40, 40))
    fbig = j3d.j3d_field_bytes(big)
    fields2 = torch.empty(fbig, dtype=torch.uint8, device="cuda")
    out2 = torch.empty(40 ** 3, dtype=torch.float64, device="cuda")
    with pytest.raises(j3d.J3DError) as e:
        j3d.j3d_solve_noalloc(big, fields2.data_ptr(), fbig, None, out2.data_ptr(), 1)
    assert e.value.status == j3d.J3D_EINVAL

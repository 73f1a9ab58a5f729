"""Caller-provided population buffers (lbm_create_ex): two device
allocations become the context's ping-pong buffers.  The run equals one
with library-allocated buffers bitwise, the current buffer holds the
documented layout (the next step pulls f_i(x) = f*_i(x - e_i) from it, or
the bounce-back f*_opp(i)(x) at a wall link), the library never frees the
buffers, and bad buffers are refused.

The buffers come from hipMalloc of the HIP runtime the library is bound to
(looked up through the library's own handle), as a torch tensor does when
torch is imported before the library loads."""
import ctypes

import numpy as np
import pytest

from paper_2505_22256_amd import workloads as W

pytestmark = pytest.mark.gpu

EX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1])
EY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1])
OPP = np.array([0, 3, 4, 1, 2, 7, 8, 5, 6])
DT = {0: np.float64, 1: np.float32}
D2H = 2  # hipMemcpyDeviceToHost


class DeviceBuffer:
    """hipMalloc / hipFree of the library's runtime."""

    def __init__(self, lbm_mod, nbytes):
        L = lbm_mod.load_library()
        L.hipMalloc.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_size_t]
        L.hipMalloc.restype = ctypes.c_int
        L.hipFree.argtypes = [ctypes.c_void_p]
        L.hipFree.restype = ctypes.c_int
        L.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
        L.hipMemcpy.restype = ctypes.c_int
        L.hipMemset.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_size_t]
        L.hipMemset.restype = ctypes.c_int
        self.L, self.n = L, nbytes
        p = ctypes.c_void_p()
        assert L.hipMalloc(ctypes.byref(p), nbytes) == 0
        self.ptr = p.value

    def read(self):
        host = np.empty(self.n, dtype=np.uint8)
        assert self.L.hipMemcpy(host.ctypes.data, self.ptr, self.n, D2H) == 0
        return host

    def free(self):
        if self.ptr:
            assert self.L.hipFree(self.ptr) == 0
            self.ptr = None


def _pair(lbm_mod, wl, storage, extra=0):
    n = lbm_mod.lbm_population_bytes(wl.nx, wl.ny, storage)
    return [DeviceBuffer(lbm_mod, n + extra) for _ in range(2)], n


def _load(lat, wl):
    lat.set_geometry(wl.solid)
    lat.set_params(wl.G_c, wl.G_ads, wl.tau)
    lat.set_body_accel(*wl.accel)
    lat.init_fields(wl.rho1, wl.rho2)


@pytest.mark.parametrize("storage", [0, 1, 2, 3])
def test_external_buffers_match_library_buffers(lbm_mod, storage):
    wl = W.random_small(21, nx=70, ny=45)
    bufs, n = _pair(lbm_mod, wl, storage)
    a = lbm_mod.Lattice(wl.nx, wl.ny, storage, wl.flags, buffers=[(d.ptr, n) for d in bufs])
    b = lbm_mod.Lattice(wl.nx, wl.ny, storage, wl.flags)
    for lat in (a, b):
        _load(lat, wl)
        lat.set_tile(64, 8, 8 if storage in (1, 2) else 0)
    for k in (1, 2, 37):
        a.step(k)
        b.step(k)
        assert np.array_equal(a.get_populations(), b.get_populations())
    a.close()
    b.close()
    # the library did not free the buffers: they are still ours to use and free
    for d in bufs:
        assert d.L.hipMemset(d.ptr, 7, d.n) == 0
        assert int(d.read()[-1]) == 7
        d.free()


@pytest.mark.parametrize("storage", [0, 1])
def test_current_buffer_holds_the_documented_layout(lbm_mod, storage):
    wl = W.random_small(22, nx=40, ny=33)
    bufs, n = _pair(lbm_mod, wl, storage)
    g = lbm_mod.Lattice(wl.nx, wl.ny, storage, wl.flags, buffers=[(d.ptr, n) for d in bufs])
    _load(g, wl)
    g.step(9)
    f = g.get_populations()  # synchronises the context's stream
    fs = bufs[g.current_buffer()].read().view(DT[storage]).astype(np.float64).reshape(2, 9, wl.ny, wl.nx)
    fluid = wl.solid == 0
    assert np.all(np.isnan(fs[:, :, ~fluid]))
    if storage == 1:  # deviations: add back w_i rho0_k, rho0_k the mean initial fluid density
        w = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
        rho0 = [wl.rho1[fluid].mean(), wl.rho2[fluid].mean()]
        fs = fs + np.array(rho0)[:, None, None, None] * w[None, :, None, None]
    pulled = np.zeros_like(fs)
    for i in range(9):
        # f*_i(x - e_i) on the doubly periodic lattice, or the bounce-back
        src = np.roll(fs[:, i], shift=(EY[i], EX[i]), axis=(1, 2))
        src_solid = np.roll(wl.solid, shift=(EY[i], EX[i]), axis=(0, 1)) == 1
        pulled[:, i] = np.where(src_solid[None], fs[:, OPP[i]], src)
    tol = 1e-15 if storage == 0 else 1e-6
    assert np.max(np.abs(f[:, :, fluid] - pulled[:, :, fluid])) <= tol
    g.close()
    for d in bufs:
        d.free()


def test_bad_external_buffers_are_refused(lbm_mod):
    wl = W.random_small(23, nx=30, ny=20)
    (a, b), n = _pair(lbm_mod, wl, lbm_mod.F32, extra=512)
    host = np.empty(n, dtype=np.uint8)
    bad = [
        ((a.ptr + 4, n), (b.ptr, n)),  # misaligned
        ((a.ptr, n - 1), (b.ptr, n - 1)),  # too small
        ((a.ptr, n), (a.ptr + 256, n)),  # overlapping
        ((host.ctypes.data, n), (b.ptr, n)),  # host memory
        ((0, n), (b.ptr, n)),  # null
    ]
    for bufs in bad:
        with pytest.raises(lbm_mod.LbmError):
            lbm_mod.Lattice(wl.nx, wl.ny, lbm_mod.F32, wl.flags, buffers=bufs)
    # a good pair still works after the refusals
    g = lbm_mod.Lattice(wl.nx, wl.ny, lbm_mod.F32, wl.flags, buffers=((a.ptr, n), (b.ptr, n)))
    _load(g, wl)
    g.step(3)
    assert g.reduce()[7] == 0
    g.close()
    a.free()
    b.free()


def test_torch_tensors_as_buffers(lbm_mod):
    """Torch tensors and a torch stream: the binding loads torch before the
    library, so both share one HIP runtime."""
    import torch
    wl = W.random_small(24, nx=70, ny=45)
    n = lbm_mod.lbm_population_bytes(wl.nx, wl.ny, lbm_mod.F32)
    ts = [torch.empty(n, dtype=torch.uint8, device="cuda") for _ in range(2)]
    a = lbm_mod.Lattice(wl.nx, wl.ny, lbm_mod.F32, wl.flags, buffers=ts)
    b = lbm_mod.Lattice(wl.nx, wl.ny, lbm_mod.F32, wl.flags)
    stream = torch.cuda.Stream()
    a.set_stream(stream.cuda_stream)
    for lat in (a, b):
        _load(lat, wl)
    a.step(20)
    b.step(20)
    assert np.array_equal(a.get_populations(), b.get_populations())
    cur = ts[a.current_buffer()].view(torch.float32).reshape(2, 9, wl.ny, wl.nx)
    solid = torch.from_numpy(wl.solid == 1).to("cuda")
    assert bool(torch.isnan(cur[:, :, solid]).all())
    a.close()
    b.close()
    ts[0].fill_(3)
    torch.cuda.synchronize()
    assert int(ts[0][5].item()) == 3


@pytest.mark.parametrize("storage", [1, 2])
def test_fluid_slots_of_the_other_buffer_are_overwritten(lbm_mod, storage):
    """The buffer that lbm_current_buffer does not name is the next step's
    output: overwriting its fluid-node slots with garbage between steps
    (solid-node slots left as the library wrote them) changes nothing,
    because the step writes every fluid slot before any step reads it."""
    import torch
    wl = W.random_small(25, nx=70, ny=45)
    n = lbm_mod.lbm_population_bytes(wl.nx, wl.ny, storage)
    ts = [torch.empty(n, dtype=torch.uint8, device="cuda") for _ in range(2)]
    a = lbm_mod.Lattice(wl.nx, wl.ny, storage, wl.flags, buffers=ts)
    b = lbm_mod.Lattice(wl.nx, wl.ny, storage, wl.flags)
    for lat in (a, b):
        _load(lat, wl)
        lat.set_tile(64, 8, 8)
    dt = torch.float32 if storage == 1 else torch.int16
    fluid = torch.from_numpy(wl.solid == 0).to("cuda")
    gen = torch.Generator(device="cuda").manual_seed(5)
    for k in (1, 2, 3, 10):
        a.synchronize()
        other = ts[a.current_buffer() ^ 1].view(dt).reshape(2, 9, wl.ny, wl.nx)
        junk = torch.randint(-30000, 30000, other.shape, generator=gen, device="cuda").to(dt)
        other[:, :, fluid] = junk[:, :, fluid]
        torch.cuda.synchronize()
        a.step(k)
        b.step(k)
        assert np.array_equal(a.get_populations(), b.get_populations()), k
    a.close()
    b.close()


def test_binding_refuses_strided_or_foreign_tensors(lbm_mod):
    """The binding hands the library one contiguous span per buffer: a
    strided view or a host tensor is refused before the library sees it."""
    import torch
    wl = W.random_small(26, nx=30, ny=20)
    n = lbm_mod.lbm_population_bytes(wl.nx, wl.ny, lbm_mod.F32)
    big = torch.empty(2 * n, dtype=torch.uint8, device="cuda")
    good = torch.empty(n, dtype=torch.uint8, device="cuda")
    with pytest.raises(ValueError):
        lbm_mod.Lattice(wl.nx, wl.ny, lbm_mod.F32, wl.flags, buffers=[big[::2], good])
    with pytest.raises(ValueError):
        lbm_mod.Lattice(wl.nx, wl.ny, lbm_mod.F32, wl.flags,
                        buffers=[torch.empty(n, dtype=torch.uint8), good])

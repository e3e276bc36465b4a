"""What tolerance the BF16 element contraction can be held to, on the CPU.

The BF16 apply splits K0 and the shifted element displacement v = u_e - s (s a
per-component translation: the element mean in the octree kernel, the values
of the element's node 0 in the uniform-brick kernel; K0 annihilates it) each
into a high and a low BF16 part (v = hi + lo + O(2^-17 |v|); the uniform-brick
kernel truncates the displacement's high part, which doubles that term) and forms
K0_hi v_hi + K0_hi v_lo + K0_lo v_hi with FP32 accumulation: the dropped
K0_lo v_lo and the two split residuals are each about 2^-18 of the product and
the FP32 sums add about 24 * 2^-24, so an element's product is good to about
3 * 2^-18 + 24 * 2^-24 = 1.3e-5 of c_e |K0| |v|.  A node sums up to eight such
products, so the apply is held to 1e-4 of max |y| (the GPU tests use that
bound).  This test emulates the two contractions in NumPy (BF16 rounding to
nearest even, FP32 accumulation) on random inputs and checks that the bound
separates them: the hi + lo form meets it with room, a hi-only form (error
about 2^-9) does not.  The emulation is test code, not the oracle."""
import numpy as np
import pytest

from oracle import element, mesh as om, system as osys

TOL = 1e-4


def bf16(x):
    """Round float32 values to BF16 (nearest, ties to even), returned as float32."""
    b = np.asarray(x, np.float32).view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32)


def bf16_trunc(x):
    """Clear the low 16 bits of float32 values (BF16 by truncation), as float32."""
    return (np.asarray(x, np.float32).view(np.uint32) & np.uint32(0xFFFF0000)).view(np.float32)


def emulated_apply(m, coef, x, lo_terms, shift="mean", hi=bf16):
    """shift: the per-component translation taken off an element's values
    before the split, the element mean (octree kernel) or its node-0 values
    (uniform-brick kernel); K0 annihilates either.  hi: how the displacement's
    high part is formed, rounded (octree kernel) or truncated (uniform-brick
    kernel; v - hi is then exact and below 2^-7 |v|)."""
    K0 = element.k0(0.3).astype(np.float32)
    Kh = bf16(K0)
    Kl = bf16(K0 - Kh)
    ed = osys.elem_dofs(m)
    ue = x.astype(np.float32)[ed].reshape(-1, 8, 3)    # (ne, 8 nodes, 3) FP32 vector entries
    ref = ue.mean(axis=1, dtype=np.float32) if shift == "mean" else ue[:, 0, :]
    v = (ue - ref[:, None, :]).reshape(-1, 24).astype(np.float32)
    vh = hi(v)
    vl = bf16(v - vh)
    y = (vh @ Kh.T).astype(np.float32)
    if lo_terms:
        y = (y + (vl @ Kh.T).astype(np.float32) + (vh @ Kl.T).astype(np.float32)).astype(np.float32)
    y = (y * coef.astype(np.float32)[:, None]).astype(np.float64)
    out = np.zeros(3 * m.n_nodes)
    np.add.at(out, ed, y)
    return out


@pytest.mark.parametrize("shift,hi", [("mean", bf16), ("node0", bf16_trunc)], ids=["octree", "uniform"])
@pytest.mark.parametrize("seed", [0, 1])
def test_bf16_tolerance_separates_hi_lo_from_hi_only(seed, shift, hi):
    rng = np.random.default_rng(seed)
    m = om.uniform_mesh((10, 6, 5))
    rho = rng.uniform(0.05, 1.0, m.n_elems)
    coef = osys.elem_coeff(m, rho)
    x = rng.uniform(-1, 1, 3 * m.n_nodes)
    exact = osys.apply_elementwise(m, coef, x.astype(np.float32).astype(np.float64))
    scale = np.abs(exact).max()
    err_split = np.abs(emulated_apply(m, coef, x, True, shift, hi) - exact).max() / scale
    err_hi = np.abs(emulated_apply(m, coef, x, False, shift, hi) - exact).max() / scale
    assert err_split <= TOL / 4, err_split
    assert err_hi >= 4 * TOL, err_hi

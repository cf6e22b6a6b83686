"""Full-size parity: the 49-qubit 7x7 grid circuit of 14 cycles, with the
benchmark's path search (best of greedy and 1024 randomised-greedy trials,
seed 1, T = 0.5), 160 GiB slicing budget and default launch configuration,
i.e. the exact kernel sequence and shapes the benchmark times (2^7 slices of
2^51.1 flops each).

The amplitude of that circuit cannot be computed by the oracle, so the
two-qubit gates are fSim(0, 0) (the identity): the network keeps its
structure (labels, path and slicing depend on gate positions only) while
every slice gets a closed-form value, the product of per-wire factors with
the sliced bonds projected (oracle/separable.py).

Error measure: |a - r| / max(|r|, 2^-(n + n_sliced)/2), the floor being the
RMS amplitude of one slice of a normalised state (a slice whose bonds
project onto nearly orthogonal states has an exact value far below what any
finite-precision contraction resolves).  Bound per precision: the 1e-5
target, or 4x the library's a-priori estimate when that is larger (it sums
u^2 (1 + log2 K) over the plan's GEMMs, u = 2^-17 for split-BF16x3, whose
estimate at this depth is 1.4e-4; 2^-21 for scaled split-FP16x3, 8.5e-6;
2^-24 for FP32).
"""

import numpy as np
import pytest

from oracle.separable import dominant_bits, separable_slice_amplitude
from workloads import grid_random_circuit, random_bitstrings

pytestmark = pytest.mark.gpu

PATH_OPTS = dict(trials=1024, seed=1, mem_budget_bytes=160.0 * 2 ** 30)   # the benchmark's plan


@pytest.fixture(scope="module")
def identity_coupled():
    import paper_2104_10523_amd as tn
    n, ops = grid_random_circuit(7, 7, 14, 2, two_qubit="fsim", fsim_params=(0.0, 0.0))
    net = tn.tn_build_network(n, ops)
    return n, ops, net, tn.tn_find_path(net, "partition", **PATH_OPTS)


@pytest.mark.parametrize("precision", ["fp32", "bf16x3", "f16x3", "auto"])
def test_rqc_7x7_14_full_size_slices(gpu, workspace, identity_coupled, precision):
    import torch
    import paper_2104_10523_amd as tn
    n, ops, net, path = identity_coupled
    ns = path.cost.n_sliced
    assert ns == 5
    floor = 2.0 ** (-(n + ns) / 2)
    rnd = random_bitstrings(1, n, 12345)[0]
    need = tn.tn_amplitudes_workspace(net, path, 2, precision)
    big = torch.empty(need, dtype=torch.uint8, device=gpu)
    tn.tn_set_workspace(big)
    # Test slices: the first ones (from slice 1 on) whose largest amplitude
    # reaches the floor.  Some slices are exactly zero (a sliced bond fixed
    # to a value the wire's state has no component on); their computed value
    # is rounding noise of the other wires' product, which can exceed the
    # floor by 10^4, so a relative error means nothing there.
    def slice_vals(s):
        return {l: (s >> (ns - 1 - i)) & 1 for i, l in enumerate(path.sliced)}
    chosen = [s for s in range(1, 2 ** ns)
              if abs(separable_slice_amplitude(n, ops, dominant_bits(n, ops, slice_vals(s)), slice_vals(s))) >= floor]
    chosen = chosen[:2] if precision == "f16x3" else chosen[:1]
    assert chosen
    try:
        # two slices for the benchmark's precision, one for the others (an
        # FP32 slice takes ~6 s per bit-string at this size)
        for s in chosen:
            vals = slice_vals(s)
            # the slice's largest amplitude (typical magnitude, so the relative
            # error means something) and one uniform bit-string
            bits = np.array([dominant_bits(n, ops, vals), rnd], dtype=np.int8)
            print(f"full-size {precision} slice {s}", flush=True)
            out, rep = tn.tn_amplitudes(net, path, bits, precision=precision, slice_begin=s, slice_count=1)
            got = out.cpu().numpy().reshape(len(bits))
            assert rep.nonfinite == 0
            tol = max(1e-5, 4 * rep.err_bound)
            for b in range(len(bits)):
                ref = separable_slice_amplitude(n, ops, bits[b], vals)
                err = abs(got[b] - ref) / max(abs(ref), floor)
                print(f"  bits {b}: got {got[b]:.6e} ref {ref:.6e} |ref|/floor {abs(ref) / floor:.2f} "
                      f"err {err:.2e} (bound {rep.err_bound:.1e}, tol {tol:.1e})", flush=True)
                assert err <= tol, (s, b, err, tol)
            assert abs(separable_slice_amplitude(n, ops, bits[0], vals)) >= floor
    finally:
        tn.tn_set_workspace(workspace)
        del big
        torch.cuda.empty_cache()

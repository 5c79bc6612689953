"""Pin of the oracle's float64 gradient on the 720p gradient window: the
256-Gaussian 32x32 sub-crop used by the GPU gradient tests, all 59 raw
parameters per Gaussian eligible, 1,000 of them drawn with a seed, central
differences with h = 1e-3 against autograd.

A parameter is left out (and counted) when one of its +-h evaluations
changes the branch signature of any pixel: the fragment set (rho^2 <=
rho_c), the core set and order, or an alpha clamp. Within one branch the
rendered colour is smooth in every raw parameter, so the difference
quotient agrees with the derivative up to O(h^2) terms."""
import math

import numpy as np
import pytest
import torch

import oracle
from tests import crops
from tests.test_oracle_grad_bins import _signature

F64 = torch.float64


@pytest.mark.slow
def test_oracle_gradient_fd_on_720p_subcrop():
    sub, cam, st, target = crops.subcrop_720p(7)
    base = [torch.tensor(x, dtype=F64) for x in sub.arrays()]
    params = [b.clone().requires_grad_(True) for b in base]
    img = oracle.render.render(*params, sub.sh_degree, cam, st, cull=False)
    # the L1 loss's weights at the unperturbed image (a fixed linear loss)
    G = torch.sign(img.detach() - torch.tensor(target, dtype=F64)) / img.numel()
    (img * G).sum().backward()
    grads = [p.grad.clone() for p in params]
    _, sig0 = _signature(base, sub.sh_degree, cam, st)
    sizes = [b.numel() for b in base]
    ends = np.cumsum(sizes)
    assert ends[-1] == 256 * 59
    rng = np.random.default_rng(1234)
    picks = rng.choice(int(ends[-1]), size=1000, replace=False)
    h = 1e-3
    gmax = [float(g.abs().max()) for g in grads]
    checked, skipped, worst = 0, 0, 0.0
    for k in picks:
        t = int(np.searchsorted(ends, k, side='right'))
        off = int(k - (ends[t] - sizes[t]))
        vals, same = [], True
        for sgn in (1, -1):
            pp = [b.clone() for b in base]
            pp[t].view(-1)[off] += sgn * h
            im, sg = _signature(pp, sub.sh_degree, cam, st)
            vals.append(float((im * G).sum()))
            same = same and sg == sig0
        if not same:
            skipped += 1
            continue
        fd = (vals[0] - vals[1]) / (2 * h)
        an = float(grads[t].view(-1)[off])
        err = abs(fd - an) / max(gmax[t], 1e-30)
        worst = max(worst, err)
        assert err <= 1e-4, (t, off, fd, an, gmax[t])
        checked += 1
    print(f"fd: {checked} checked, {skipped} branch changes left out, worst {worst:.2e}")
    assert checked >= 900, (checked, skipped)

"""GPU RMS loss and its gradient against the FP64 reference (FP64 sums in another order: the loss
within 1e-12 relative, the float32 gradient within 2 ulp)."""
import numpy as np
import pytest

import oracle as O
from helpers import DEV, afr_mod, torch_mod

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("shape,scale", [((3, 64, 64), 1.0), ((3, 480, 640), 1.0 / 32),
                                         ((3, 7, 5), 2.5), ((1000003,), 1.0)])
def test_rms_loss_matches_reference(shape, scale):
    torch = torch_mod()
    afr = afr_mod()
    rng = np.random.default_rng(sum(shape))
    img = rng.random(shape).astype(np.float32)
    ref = (img + rng.normal(0, 0.05, shape)).astype(np.float32)
    loss, grad = afr.rms_loss(torch.from_numpy(img).to(DEV), torch.from_numpy(ref).to(DEV), scale)
    np.testing.assert_allclose(loss.item(), scale * O.rms(img, ref), rtol=1e-12)
    np.testing.assert_allclose(grad.cpu().numpy(), O.rms_grad(img, ref, scale), rtol=3e-7, atol=1e-30)


def test_rms_loss_of_equal_images_is_zero_with_zero_gradient():
    torch = torch_mod()
    afr = afr_mod()
    img = torch.rand((3, 33, 17), device=DEV)
    loss, grad = afr.rms_loss(img, img.clone(), 1.0)
    assert loss.item() == 0.0 and bool((grad == 0).all().item())
    loss, grad = afr.rms_loss(torch.zeros(0, device=DEV), torch.zeros(0, device=DEV), 1.0)
    assert loss.item() == 0.0 and grad.numel() == 0

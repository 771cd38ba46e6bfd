"""Host checks of the network module: the 3x3x3 convolution computed as a 2-D convolution
equals torch's 3-D convolution (forward and gradients), on the CPU."""
import pytest

torch = pytest.importorskip("torch")
N = pytest.importorskip("paper_2201_02309_amd.network")


@pytest.mark.parametrize("cin,cout,shape", [(1, 16, (2, 5, 6, 7)), (16, 16, (1, 4, 3, 9)),
                                            (16, 1, (1, 1, 5, 5))])
def test_conv3x3x3_equals_conv3d(cin, cout, shape):
    torch.manual_seed(0)
    m = N.Conv3x3x3(cin, cout).double()
    B, D, H, W = shape
    x = torch.randn(B, cin, D, H, W, dtype=torch.float64, requires_grad=True)
    y = m(x)
    ref = torch.nn.functional.conv3d(x, m.weight, m.bias, padding=1)
    assert torch.allclose(y, ref, rtol=0, atol=1e-12)
    g = torch.randn_like(y)
    gx, gw, gb = torch.autograd.grad(y, (x, m.weight, m.bias), g)
    rx, rw, rb = torch.autograd.grad(ref, (x, m.weight, m.bias), g)
    for a, b in ((gx, rx), (gw, rw), (gb, rb)):
        assert torch.allclose(a, b, rtol=0, atol=1e-10)


def test_subnet_shapes_and_residual():
    torch.manual_seed(1)
    net = N.SubNet(channels=4, blocks=3)
    x = torch.randn(1, 1, 3, 5, 6)
    with torch.no_grad():
        net.out.weight.zero_()
        net.out.bias.zero_()
    assert torch.equal(net(x), x)                 # zero last convolution: identity skip

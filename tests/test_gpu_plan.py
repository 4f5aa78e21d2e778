"""The automatic launch plan (tile shape, z-chunk, work-groups) for grids
whose best plan was measured on MI355X (256 CUs): every entry below is the
fastest configuration, or within 3 % of it, found by timing every tile
shape and chunk count for that grid.  A change of the planner that moves
one of them has to be measured again."""
import pytest
import torch

pytestmark = pytest.mark.gpu

# (nx, ny, nz, dtype): (tile variant, z-chunk, work-groups)
PLANS = {
    (512, 512, 512, "f32"): ("t256x8_r1", 256, 256),      # one round of 256 x 8 tiles
    (512, 512, 512, "f16"): ("t128x16_r2", 128, 512),     # 256-thread groups, two per CU
    (512, 512, 512, "f16uv"): ("t128x32_r2", 128, 256),
    (755, 994, 1000, "f32"): ("t256x8_r1", 500, 750),     # the paper's largest shape
    (320, 320, 256, "f32"): ("t128x16_r1", 64, 240),      # narrow: 256-wide tiles idle lanes
    (600, 600, 1000, "f32"): ("t128x16_r1", 1000, 190),   # one chunk: a second round costs more
    (400, 400, 400, "f32"): ("t128x16_r1", 80, 500),      # two full rounds beat 78 % of one
    (200, 200, 1000, "f32"): ("t256x8_r1", 100, 250),     # one tile wide: equal tiles beat 128 x 16
    (192, 192, 512, "f32"): ("t256x8_r1", 52, 240),
    (128, 512, 256, "f32"): ("t128x16_r1", 32, 256),      # 128 wide: 256-wide tiles idle half the lanes
    (64, 64, 64, "f32"): ("t64x16_r1", 1, 256),           # small grid: latency-bound plan
}


@pytest.mark.parametrize("shape", sorted(PLANS), ids=lambda s: "x".join(map(str, s[:3])) + "-" + s[3])
def test_automatic_plan(wave_mod, shape):
    if torch.cuda.get_device_properties(0).multi_processor_count != 256:
        pytest.skip("the expected plans were measured on a 256-CU MI355X")
    nx, ny, nz, dtype = shape
    print(f"case: plan {nx}x{ny}x{nz} {dtype}", flush=True)
    k = torch.full((1, 1, 1), 2.0, dtype=torch.float32, device="cuda").expand(nz, ny, nx)
    prop = wave_mod.Propagator(nx, ny, nz, (10.0, 10.0, 10.0), k, src=(nz // 2, ny // 2, nx // 2),
                               dtype=dtype)
    v, zc, wg = prop.config()
    prop.close()
    del prop
    torch.cuda.empty_cache()
    assert (wave_mod.wave_variant_name(v), zc, wg) == PLANS[shape]

"""The pins catch planted mistakes.

Each case copies the oracle's source, plants one plausible mistake (a dropped factor, a
swapped index, a transposed size, a missing term of the adjoint), builds the copy with
gcc into a temporary directory and runs the pin that is meant to catch it against that
build: the pin must fail.  The real oracle passes the same pins elsewhere in the suite.
"""
import os

import numpy as np
import pytest

from oracle import oracle as O

from . import test_oracle_pins as P
from . import test_oracle_pins_brdf2 as PB
from . import test_oracle_pins_camera as PC
from . import test_oracle_pins_camera_edges as PE
from . import test_oracle_pins_lights as PL

SRC = open(O.SRC).read()

# (name, text in the oracle, planted replacement, the pin that must fail)
MUTANTS = [
    ("environment NEE without its pi",
     "double es = d->nmap_sample ? PI * fb.c / dot(nss, we) : PI;",
     "double es = d->nmap_sample ? PI * fb.c / dot(nss, we) : 1.0;",
     lambda: PL.test_environment_on_a_lambert_plane(1)),
    ("environment added on escaped bounce rays",
     "if (depth == 0)\n                for (int c = 0; c < 3; ++c) L[c] += beta[c] * d->env[c];",
     "if (depth >= 0)\n                for (int c = 0; c < 3; ++c) L[c] += beta[c] * d->env[c];",
     lambda: PL.test_environment_on_a_lambert_plane(3)),
    ("environment shadow ray ignored",
     "int occ = occluded(d, &cx->sc, x, we, 1e300, prim, &mo);",
     "int occ = 0 * occluded(d, &cx->sc, x, we, 1e300, prim, &mo);",
     PL.test_environment_occlusion_under_a_ceiling),
    ("projector lookup with u and v swapped",
     "bilinear_at(pu - 0.5, pv - 0.5, d->Wp, d->Hp)",
     "bilinear_at(pv - 0.5, pu - 0.5, d->Wp, d->Hp)",
     lambda: PL.test_projector_lookup_with_a_non_constant_image(0.0, 40, 24)),
    ("projector lookup without the half-texel offset",
     "bilinear_at(pu - 0.5, pv - 0.5, d->Wp, d->Hp)",
     "bilinear_at(pu, pv, d->Wp, d->Hp)",
     lambda: PL.test_projector_lookup_with_a_non_constant_image(0.0, 40, 24)),
    ("projector lookup with W_p and H_p transposed",
     "bilinear_at(pu - 0.5, pv - 0.5, d->Wp, d->Hp)",
     "bilinear_at(pu - 0.5, pv - 0.5, d->Hp, d->Wp)",
     lambda: PL.test_projector_lookup_with_a_non_constant_image(0.0, 17, 29)),
    ("projector NEE after a bounce without the path throughput",
     "L[c] += beta[c] * fb.f[c] * E[c] * geom;",
     "L[c] += fb.f[c] * E[c] * geom;",
     PL.test_integrating_sphere),
    ("projector intensity without 1/cos^3",
     "double geom = fb.c / (ca * ca * ca * dist * dist);",
     "double geom = fb.c / (dist * dist);",
     PL.test_integrating_sphere),
    ("adjoint: environment terms dropped",
     "S[1][c] = d->env[c] * v->es;",
     "S[1][c] = 0.0 * v->es;",
     lambda: P.test_adjoint_matches_central_differences(False, 0.4)),
    ("adjoint: roughness terms dropped",
     "gr += bd * b->dfr[c] * cs;",
     "gr += 0.0 * cs;",
     lambda: P.test_adjoint_matches_central_differences(False, 0.4)),
    ("metallic does not scale the diffuse lobe",
     "b.f[c] = (1.0 - mu) * a[c] / PI + F * DGw;",
     "b.f[c] = a[c] / PI + F * DGw;",
     PB.test_metallic_peak_at_normal_incidence),
    ("metallic does not tint the Fresnel reflectance",
     "double F0 = (1.0 - mu) * (0.08 * sp) + mu * a[c];",
     "double F0 = 0.08 * sp;",
     PB.test_metallic_peak_at_normal_incidence),
    ("normal-map frame with the wrong handedness",
     "*B = cross(n, *T);",
     "*B = cross(*T, n);",
     lambda: PB.test_normal_map_tilts_the_shading_normal_on_a_plane(False)),
    ("normal map read without decoding 2 v - 1",
     "v3 t = mk(2.0 * v[0] - 1.0, 2.0 * v[1] - 1.0, 2.0 * v[2] - 1.0);",
     "v3 t = mk(v[0], v[1], v[2]);",
     lambda: PB.test_normal_map_tilts_the_shading_normal_on_a_plane(False)),
    ("projector cosine about the geometric normal under a normal map",
     "double geom = fb.c / (ca * ca * ca * dist * dist);",
     "double geom = cp / (ca * ca * ca * dist * dist);",
     lambda: PB.test_normal_map_tilts_the_shading_normal_on_a_plane(True)),
    ("adjoint: normal cotangent not projected onto the unit sphere",
     "v3 gt = scl(sub(gl, scl(v->th, dot(v->th, gl))), 1.0 / v->tlen);",
     "v3 gt = scl(gl, 1.0 / v->tlen);",
     PB.test_adjoint_on_metallic_and_normal_map_matches_central_differences),
    ("adjoint: metallic terms dropped",
     "gm += bd * b->dfm[c] * cs;",
     "gm += 0.0 * cs;",
     PB.test_adjoint_on_metallic_and_normal_map_matches_central_differences),
    ("adjoint: cosine derivative missing from the normal cotangent",
     "b.dfcn[c] = add(scl(wi, (1.0 - mu) * a[c] / PI), scl(dS, F));",
     "b.dfcn[c] = scl(dS, F);",
     PB.test_adjoint_on_metallic_and_normal_map_matches_central_differences),
    ("camera pose: camera centre +R^T t instead of -R^T t",
     "v3 o = scl(mattv(Rc, mk(tc[0], tc[1], tc[2])), -1.0);",
     "v3 o = scl(mattv(Rc, mk(tc[0], tc[1], tc[2])), 1.0);",
     PC.test_camera_pose_gradient_on_a_lit_plane),
    ("camera pose: projector term without the 1/cos^3 falloff",
     "out[c] += fb.f[c] * fb.c * E[c] / (ca * ca * ca * dist * dist);",
     "out[c] += fb.f[c] * fb.c * E[c] / (dist * dist);",
     PC.test_camera_pose_gradient_on_a_lit_plane),
    ("camera pose: bounce term dropped",
     "out[c] += fb.f[c] * fb.c * Sb[c];",
     "out[c] += 0.0 * Sb[c];",
     PC.test_camera_pose_gradient_through_the_bounce),
    ("camera edges: jump taken as f+ - f-",
     "for (int ch = 0; ch < 3; ++ch) J += g[ch] * (f[0][ch] - f[1][ch]);",
     "for (int ch = 0; ch < 3; ++ch) J += g[ch] * (f[1][ch] - f[0][ch]);",
     PE.test_square_silhouette_constant_cotangent),
    ("camera edges: image parameter used as the 3D parameter",
     "double mu = lam * c.wA / (lam * c.wA + (1.0 - lam) * c.wB);",
     "double mu = lam;",
     PE.test_square_silhouette_constant_cotangent),
    ("camera edges: speed without the perspective division's x term",
     "double ci_x = (d->Kc[r] - x * d->Kc[6 + r]) / h.z;",
     "double ci_x = d->Kc[r] / h.z;",
     PE.test_square_silhouette_constant_cotangent),
    ("camera edges: sample weight without the segment length",
     "J *= c.len / (double)n;",
     "J *= 1.0 / (double)n;",
     PE.test_square_silhouette_constant_cotangent),
    ("camera edges: pixel indices transposed",
     "const double* g = dE + 3 * ((size_t)pj * d->Wc + pi);",
     "const double* g = dE + 3 * ((size_t)pi * d->Wc + pj);",
     PE.test_square_silhouette_random_cotangent),
    ("camera edges: faces at an angle not taken",
     "if (len(cross(n0, n1)) > 1e-9) return 1;",
     "if (len(cross(n0, n1)) > 1e9) return 1;",
     PE.test_box_of_one_emission_without_seams),
    ("camera edges: faces folded flat not taken",
     "dot(sub(C1, A), sub(B, A)) / dot(sub(B, A), sub(B, A)) > 0)",
     "dot(sub(C1, A), sub(B, A)) / dot(sub(B, A), sub(B, A)) > 1e300)",
     PE.test_faces_folded_flat),
    ("camera edges: texture seams not taken",
     "if (u0[2 * a0] != u1[2 * a1] || u0[2 * a0 + 1] != u1[2 * a1 + 1] || u0[2 * b0] != u1[2 * b1] ||",
     "if (0 && (u0[2 * a0] != u1[2 * a1] || u0[2 * a0 + 1] != u1[2 * a1 + 1] || u0[2 * b0] != u1[2 * b1]) &&",
     PE.test_texture_seam_under_the_environment),
    ("camera edges: emission seams not taken",
     "if (d->Le[3 * e->f0 + c] != d->Le[3 * e->f1 + c]) return 1;",
     "if (0 * d->Le[3 * e->f0 + c] != 0) return 1;",
     PE.test_emission_seam_and_flat_fold),
    ("camera edges: no welding of repeated vertices",
     "canon[v[i].i] = same ? canon[v[i - 1].i] : v[i].i;",
     "canon[v[i].i] = v[i].i + 0 * same;",
     PE.test_closed_box),
    ("camera edges: faces of no area kept",
     "    return m.x != 0 || m.y != 0 || m.z != 0;",
     "    return 1 || m.x != 0 || m.y != 0 || m.z != 0;",
     PE.test_faces_of_no_area_take_no_part),
    ("camera edges: no clipping at the camera plane",
     "if (hA.z < wmin) s0 = (wmin - hA.z) / (hB.z - hA.z);",
     "if (0) s0 = (wmin - hA.z) / (hB.z - hA.z);",
     PE.test_floor_reaching_behind_the_camera),
]


@pytest.mark.parametrize("name,orig,planted,pin", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pin_catches_planted_mistake(tmp_path, name, orig, planted, pin):
    assert SRC.count(orig) == 1, f"the text to mutate is not unique in the oracle: {orig!r}"
    src = os.path.join(tmp_path, "mutant.c")
    with open(src, "w") as f:
        f.write(SRC.replace(orig, planted))
    lib = O.build(force=True, src=src, out=os.path.join(tmp_path, "libmutant.so"))
    with O.library(lib):
        with pytest.raises(AssertionError):
            with np.errstate(all="ignore"):
                pin()

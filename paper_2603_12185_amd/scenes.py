"""Seeded synthetic scene generators.

This module produces model descriptions and initial states as plain numpy
arrays.  It holds none of the contact method's arithmetic: it only places
bodies, draws sizes, masses, friction coefficients and initial velocities,
and is the single source of inputs shared by the GPU library and the CPU
oracle.  Every floating constant is rounded to a value that float32 represents
exactly, so both sides simulate exactly the same model.

Scene dictionary keys (shapes use nw = worlds, nb = bodies, ng = geoms):

  nworld, nbody, ngeom, ncon_max, condim          ints
  body_parent[nb], body_jnt[nb]                   int32 (parent -1 = world)
  body_pos[nb,3], body_quat[nb,4]                 body frame in parent frame at q = 0
  body_ipos[nb,3]                                 centre of mass in the body frame
  jnt_axis[nb,3]                                  hinge/slide axis in the body frame
  body_mass[nw,nb], body_inertia[nw,nb,3]         principal inertia about the COM
  geom_type[ng], geom_body[ng]                    int32 (body -1 = static)
  geom_size[nw,ng,3], geom_pos[nw,ng,3], geom_quat[nw,ng,4], geom_friction[nw,ng,3]
  h, gravity[3], k_user, d_user, solimp[5], margin
  q0[nw,nq], v0[nw,nv]                            float32 initial state

Quaternions are (w, x, y, z).  Free joints use q = (COM position, orientation)
and v = (COM linear velocity, angular velocity), both in world coordinates.
"""
from __future__ import annotations

import math

import numpy as np

PLANE, SPHERE, CAPSULE, BOX = 0, 1, 2, 3
JNT_FREE, JNT_HINGE, JNT_SLIDE = 0, 1, 2

# Impedance shape defaults (r_min, r_max, width, midpoint, power) printed in
# the paper's impedance heuristic section.
SOLIMP_DEFAULT = (0.9, 0.95, 0.001, 0.5, 2.0)

_QPOS = {JNT_FREE: 7, JNT_HINGE: 1, JNT_SLIDE: 1}
_QVEL = {JNT_FREE: 6, JNT_HINGE: 1, JNT_SLIDE: 1}


def f32(x):
    """Round to the nearest float32 and return float64 (exactly representable)."""
    return np.asarray(x, dtype=np.float32).astype(np.float64)


def dims(scene) -> tuple[int, int]:
    """(nq, nv) of a scene from its joint types."""
    jt = scene["body_jnt"]
    return int(sum(_QPOS[int(t)] for t in jt)), int(sum(_QVEL[int(t)] for t in jt))


def nfacet(condim: int) -> int:
    return {1: 1, 3: 4, 4: 6, 6: 10}[int(condim)]


def _quat_to_mat(qt):
    w, x, y, z = qt / np.linalg.norm(qt)
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
    ])


def _quat_z_to(nrm):
    """A unit quaternion whose rotation maps +z onto the unit vector nrm."""
    nrm = np.asarray(nrm, float) / np.linalg.norm(nrm)
    z = np.array([0.0, 0.0, 1.0])
    c = float(np.dot(z, nrm))
    if c > 1 - 1e-12:
        return np.array([1.0, 0.0, 0.0, 0.0])
    if c < -1 + 1e-12:
        return np.array([0.0, 1.0, 0.0, 0.0])
    ax = np.cross(z, nrm)
    ax /= np.linalg.norm(ax)
    ang = math.acos(c)
    return np.array([math.cos(ang / 2), *(math.sin(ang / 2) * ax)])


class _Builder:
    """Accumulates bodies and geoms of one model shared by nworld worlds."""

    def __init__(self, nworld=1):
        self.nworld = nworld
        self.bodies = []   # dicts
        self.geoms = []    # dicts

    def body(self, jnt, parent=-1, pos=(0, 0, 0), quat=(1, 0, 0, 0), ipos=(0, 0, 0),
             axis=(0, 0, 1), mass=1.0, inertia=(1, 1, 1)):
        """mass / inertia may be scalars/3-vectors or per-world arrays."""
        self.bodies.append(dict(jnt=jnt, parent=parent, pos=pos, quat=quat, ipos=ipos,
                                axis=axis, mass=mass, inertia=inertia))
        return len(self.bodies) - 1

    def geom(self, gtype, body=-1, size=(0, 0, 0), pos=(0, 0, 0), quat=(1, 0, 0, 0),
             friction=(0, 0, 0)):
        """size / friction may be per-world arrays [nw,3]."""
        self.geoms.append(dict(type=gtype, body=body, size=size, pos=pos, quat=quat,
                               friction=friction))
        return len(self.geoms) - 1

    def build(self, *, condim=3, h=0.002, k_user=0.1, d_user=0.001, solimp=SOLIMP_DEFAULT,
              margin=0.0, gravity=(0, 0, -9.81), ncon_max=64, name="scene"):
        nw, nb, ng = self.nworld, len(self.bodies), len(self.geoms)

        def per_world(val, width):
            a = np.asarray(val, dtype=np.float64)
            if a.ndim == 0:
                a = np.full((nw, width), float(a)) if width > 1 else np.full((nw,), float(a))
            elif width > 1 and a.shape == (width,):
                a = np.broadcast_to(a, (nw, width))
            elif width == 1 and a.shape == ():
                a = np.full((nw,), float(a))
            return np.array(a, dtype=np.float64)

        def gstack(key, width):
            if ng == 0:
                return np.zeros((nw, 0, width))
            return f32(np.stack([per_world(g[key], width) for g in self.geoms], axis=1))

        s = dict(
            name=name, nworld=nw, nbody=nb, ngeom=ng, ncon_max=int(ncon_max), condim=int(condim),
            body_parent=np.array([b["parent"] for b in self.bodies], np.int32).reshape(nb),
            body_jnt=np.array([b["jnt"] for b in self.bodies], np.int32).reshape(nb),
            body_pos=f32(np.array([b["pos"] for b in self.bodies], float).reshape(nb, 3)),
            body_quat=f32(np.array([b["quat"] for b in self.bodies], float).reshape(nb, 4)),
            body_ipos=f32(np.array([b["ipos"] for b in self.bodies], float).reshape(nb, 3)),
            jnt_axis=f32(np.array([b["axis"] for b in self.bodies], float).reshape(nb, 3)),
            body_mass=f32(np.stack([per_world(b["mass"], 1) for b in self.bodies], axis=1)
                          .reshape(nw, nb)) if nb else np.zeros((nw, 0)),
            body_inertia=f32(np.stack([per_world(b["inertia"], 3) for b in self.bodies], axis=1)
                             .reshape(nw, nb, 3)) if nb else np.zeros((nw, 0, 3)),
            geom_type=np.array([g["type"] for g in self.geoms], np.int32).reshape(ng),
            geom_body=np.array([g["body"] for g in self.geoms], np.int32).reshape(ng),
            geom_size=gstack("size", 3), geom_pos=gstack("pos", 3),
            geom_quat=gstack("quat", 4), geom_friction=gstack("friction", 3),
            h=float(f32(h)), gravity=f32(np.array(gravity, float)),
            k_user=float(f32(k_user)), d_user=float(f32(d_user)),
            solimp=f32(np.array(solimp, float)), margin=float(f32(margin)),
        )
        nq, nv = dims(s)
        s["q0"] = np.zeros((nw, nq), np.float32)
        s["v0"] = np.zeros((nw, nv), np.float32)
        # default state: free bodies at their body_pos/body_quat, joints at 0
        qa = 0
        for b in range(nb):
            if s["body_jnt"][b] == JNT_FREE:
                s["q0"][:, qa:qa + 3] = s["body_pos"][b]
                s["q0"][:, qa + 3:qa + 7] = s["body_quat"][b]
            qa += _QPOS[int(s["body_jnt"][b])]
        return s


def qadr(scene):
    """Start index in q of each body's joint."""
    out, a = [], 0
    for t in scene["body_jnt"]:
        out.append(a)
        a += _QPOS[int(t)]
    return np.array(out, np.int64)


def dadr(scene):
    """Start index in v of each body's joint."""
    out, a = [], 0
    for t in scene["body_jnt"]:
        out.append(a)
        a += _QVEL[int(t)]
    return np.array(out, np.int64)


def _random_quat(rng):
    q = rng.standard_normal(4)
    return q / np.linalg.norm(q)


# --------------------------------------------------------------------------
# Benchmark-shaped scenes
# --------------------------------------------------------------------------

def boxes_drop(seed=0, k_user=0.1, d_user=0.001, condim=3, ncon_max=64):
    """One world: 8 free boxes (edge 0.1 m, 1 kg) dropped onto a ground plane.

    Boxes sit on a 2 x 4 grid with 0.3 m spacing (they never touch each other),
    random orientations (normalised 4-vector of N(0,1)), lowest-corner clearance
    U(0.05, 0.3) m, zero initial velocity, box friction U(0.3, 1.0); the ground
    has zero friction so the pair friction is the box's.
    """
    rng = np.random.default_rng([seed, 1])
    half, mass = 0.05, 1.0
    inertia = mass * (2 * half) ** 2 / 6.0
    b = _Builder(1)
    b.geom(PLANE, -1, friction=(0, 0, 0))
    xs, ys = (-0.45, -0.15, 0.15, 0.45), (-0.15, 0.15)
    poses = []
    for iy in range(2):
        for ix in range(4):
            qt = _random_quat(rng)
            clearance = rng.uniform(0.05, 0.3)
            R = _quat_to_mat(qt)
            corners = np.array([[sx, sy, sz] for sz in (-1, 1) for sy in (-1, 1)
                                for sx in (-1, 1)], float) * half
            low = min((R @ c)[2] for c in corners)
            mu = rng.uniform(0.3, 1.0)
            bi = b.body(JNT_FREE, mass=mass, inertia=(inertia,) * 3)
            b.geom(BOX, bi, size=(half, half, half), friction=(mu, 0.005, 0.0005))
            poses.append((xs[ix], ys[iy], clearance - low, qt))
    s = b.build(condim=condim, k_user=k_user, d_user=d_user, ncon_max=ncon_max,
                name="boxes_drop")
    for i, (x, y, z, qt) in enumerate(poses):
        s["q0"][0, 7 * i:7 * i + 3] = (x, y, z)
        s["q0"][0, 7 * i + 3:7 * i + 7] = qt
    return s


def dense_pile(nworld=4096, nsphere=64, seed=0, k_user=0.1, d_user=0.001, condim=3,
               ncon_max=1024, walls=True):
    """Spheres in a 0.5 m walled box, one independent random stream per world.

    Ground z = 0 and (optionally) four walls at x, y = +-0.25 with inward
    normals, all frictionless and static.  Spheres: radius U(0.02, 0.05) m,
    density 1000 kg/m^3, solid-sphere inertia, friction U(0.3, 1.0) (torsional
    U(1, 5) mm, rolling U(0.1, 0.5) mm, used when condim >= 4).  Centres start on
    a 4 x 4 x (nsphere/16) lattice with 0.11 m pitch, centred in x/y, z = 0.06 +
    0.11 i, jittered by U(+-5 mm); linear velocities N(0, 1e-3) m/s.
    """
    assert nsphere % 16 == 0, "nsphere must be a multiple of 16 (4 x 4 layers)"
    nlay = nsphere // 16
    rad = np.empty((nworld, nsphere))
    mu = np.empty((nworld, nsphere, 3))
    pos = np.empty((nworld, nsphere, 3))
    vel = np.empty((nworld, nsphere, 3))
    grid = np.array([[ix, iy, iz] for iz in range(nlay) for iy in range(4) for ix in range(4)],
                    float)
    base = np.stack([(grid[:, 0] - 1.5) * 0.11, (grid[:, 1] - 1.5) * 0.11,
                     0.06 + 0.11 * grid[:, 2]], axis=1)
    for w in range(nworld):
        rng = np.random.default_rng([seed, 2, w])
        rad[w] = rng.uniform(0.02, 0.05, nsphere)
        mu[w, :, 0] = rng.uniform(0.3, 1.0, nsphere)
        mu[w, :, 1] = rng.uniform(0.001, 0.005, nsphere)
        mu[w, :, 2] = rng.uniform(0.0001, 0.0005, nsphere)
        pos[w] = base + rng.uniform(-0.005, 0.005, (nsphere, 3))
        vel[w] = rng.normal(0.0, 1e-3, (nsphere, 3))
    rad = f32(rad)
    mass = f32(1000.0 * 4.0 / 3.0 * np.pi * rad ** 3)
    inert = f32(0.4 * mass * rad ** 2)
    b = _Builder(nworld)
    b.geom(PLANE, -1)
    if walls:
        for nrm, p in (((1, 0, 0), (-0.25, 0, 0)), ((-1, 0, 0), (0.25, 0, 0)),
                       ((0, 1, 0), (0, -0.25, 0)), ((0, -1, 0), (0, 0.25, 0))):
            b.geom(PLANE, -1, pos=p, quat=_quat_z_to(nrm))
    for i in range(nsphere):
        bi = b.body(JNT_FREE, mass=mass[:, i],
                    inertia=np.repeat(inert[:, i:i + 1], 3, axis=1))
        b.geom(SPHERE, bi, size=np.stack([rad[:, i], np.zeros(nworld), np.zeros(nworld)], 1),
               friction=mu[:, i, :])
    s = b.build(condim=condim, k_user=k_user, d_user=d_user, ncon_max=ncon_max,
                name=f"dense_pile_{nworld}x{nsphere}")
    q = s["q0"].reshape(nworld, nsphere, 7)
    q[:, :, 0:3] = pos
    q[:, :, 3] = 1.0
    q[:, :, 4:7] = 0.0
    s["v0"].reshape(nworld, nsphere, 6)[:, :, 0:3] = vel
    return s


# --------------------------------------------------------------------------
# Small scenes used by the closed-form and parity tests
# --------------------------------------------------------------------------

def sphere_on_plane(nworld=1, radius=0.05, mass=1.0, mu=(0.5, 0.0, 0.0), condim=3,
                    k_user=0.1, d_user=0.001, z0=None, h=0.002, gravity=(0, 0, -9.81),
                    solimp=SOLIMP_DEFAULT, ncon_max=8):
    b = _Builder(nworld)
    b.geom(PLANE, -1)
    bi = b.body(JNT_FREE, pos=(0, 0, radius if z0 is None else z0), mass=mass,
                inertia=(0.4 * mass * radius ** 2,) * 3)
    b.geom(SPHERE, bi, size=(radius, 0, 0), friction=mu)
    return b.build(condim=condim, k_user=k_user, d_user=d_user, h=h, gravity=gravity,
                   solimp=solimp, ncon_max=ncon_max, name="sphere_on_plane")


def point_mass(mu=0.5, radius=0.05, mass=1.0, z0=None, condim=3, k_user=0.1, d_user=0.001,
               h=0.002, ncon_max=8):
    """A point mass moved by three slide joints (x, y, z) with a sphere geom on a plane.

    The two intermediate slide bodies are massless; all mass sits on the last body,
    so the mass matrix is m*I3 and the body never rotates.
    """
    b = _Builder(1)
    b.geom(PLANE, -1)
    b0 = b.body(JNT_SLIDE, -1, axis=(1, 0, 0), mass=0.0, inertia=(0, 0, 0))
    b1 = b.body(JNT_SLIDE, b0, axis=(0, 1, 0), mass=0.0, inertia=(0, 0, 0))
    b2 = b.body(JNT_SLIDE, b1, axis=(0, 0, 1), mass=mass, inertia=(1e-3, 1e-3, 1e-3))
    b.geom(SPHERE, b2, size=(radius, 0, 0), friction=(mu, 0, 0))
    s = b.build(condim=condim, k_user=k_user, d_user=d_user, h=h, ncon_max=ncon_max,
                name="point_mass")
    s["q0"][0, 2] = radius if z0 is None else z0
    return s


def pendulum(length=0.5, mass=1.0, radius=0.02, gravity=(0, 0, -9.81), h=0.002):
    """Hinge about world y at the origin, point-like bob at (0, 0, -length)."""
    b = _Builder(1)
    i = 0.4 * mass * radius ** 2
    bi = b.body(JNT_HINGE, -1, axis=(0, 1, 0), ipos=(0, 0, -length), mass=mass,
                inertia=(i, i, i))
    b.geom(SPHERE, bi, size=(radius, 0, 0), pos=(0, 0, -length))
    return b.build(gravity=gravity, h=h, name="pendulum")


def hinge_bob_on_plane(length=0.3, mass=0.8, radius=0.03, inertia=(2e-3, 3e-3, 1e-3), angle=0.4,
                       depth=0.001, mu=(0.6, 0.004, 0.0004), condim=3, k_user=0.1, d_user=0.001,
                       gravity=(0, 0, -9.81), h=0.002, ncon_max=8):
    """A hinge about world y at (0, 0, z_h) holding a sphere bob at distance
    `length` (COM and sphere centre at angle `angle` from straight down), z_h
    chosen so that the sphere reaches `depth` into the ground plane."""
    b = _Builder(1)
    b.geom(PLANE, -1)
    zh = length * math.cos(angle) + radius - depth
    bi = b.body(JNT_HINGE, -1, pos=(0, 0, zh), axis=(0, 1, 0), ipos=(0, 0, -length), mass=mass,
                inertia=inertia)
    b.geom(SPHERE, bi, size=(radius, 0, 0), pos=(0, 0, -length), friction=mu)
    s = b.build(condim=condim, k_user=k_user, d_user=d_user, h=h, gravity=gravity, ncon_max=ncon_max,
                name="hinge_bob_on_plane")
    # a positive rotation about +y takes -z toward -x
    s["q0"][0, 0] = angle
    return s


def sibling_sliders(nworld=1, seed=0, radius=0.03, overlap=0.002, mu=(0.6, 0.004, 0.0004), condim=3,
                    k_user=0.1, d_user=0.001, gravity=(0, 0, 0), carrier="slide", axis2=(0, 1, 0),
                    ncon_max=8):
    """A carrier body (a slide along x, or a free joint) with two children
    that slide along y (the second along `axis2`), each carrying a sphere; the
    spheres overlap along x by `overlap`, so their contact joins two bodies of
    one subtree (siblings, not parent and child).  World 0 has masses 0.7
    (carrier), 0.3 and 0.5 and the velocities below; further worlds draw
    masses and velocities (seeded)."""
    rng = np.random.default_rng([seed, 13])
    m = np.tile([0.7, 0.3, 0.5], (nworld, 1))
    m[1:] = rng.uniform(0.2, 1.0, (nworld - 1, 3))
    b = _Builder(nworld)
    jc = JNT_SLIDE if carrier == "slide" else JNT_FREE
    c = b.body(jc, -1, pos=(0, 0, 0.2), axis=(1, 0, 0), mass=m[:, 0],
               inertia=np.stack([m[:, 0] * 4e-3, m[:, 0] * 5e-3, m[:, 0] * 6e-3], 1))
    for k, x, ax in ((1, 0.0, (0, 1, 0)), (2, 2 * radius - overlap, axis2)):
        bk = b.body(JNT_SLIDE, c, pos=(x, 0, 0), axis=ax, mass=m[:, k],
                    inertia=np.repeat((0.4 * m[:, k] * radius * radius)[:, None], 3, 1))
        b.geom(SPHERE, bk, size=(radius, 0, 0), friction=mu)
    s = b.build(condim=condim, k_user=k_user, d_user=d_user, gravity=gravity, ncon_max=ncon_max,
                name="sibling_sliders")
    da = dadr(s)
    for w in range(nworld):
        v = s["v0"][w]
        if w == 0:
            v[da[0]:da[1]] = (0.05, 0.0, 0.0, 0.3, -0.2, 0.7)[:da[1] - da[0]]
            v[da[1]], v[da[2]] = 0.04, -0.03
        else:
            v[da[0]:da[1]] = rng.normal(0, 0.1, da[1] - da[0])
            v[da[1]], v[da[2]] = rng.normal(0, 0.05, 2)
    return s


def double_pendulum(l1=0.6, lc1=0.3, lc2=0.25, m1=1.3, m2=0.7, i1=(0.02, 0.03, 0.01),
                    i2=(0.015, 0.01, 0.02), gravity=(0, 0, -9.81)):
    """Planar two-link arm in the x-z plane, hinges about y; angles measured from +x."""
    b = _Builder(1)
    b0 = b.body(JNT_HINGE, -1, axis=(0, -1, 0), ipos=(lc1, 0, 0), mass=m1, inertia=i1)
    b.body(JNT_HINGE, b0, pos=(l1, 0, 0), axis=(0, -1, 0), ipos=(lc2, 0, 0), mass=m2,
           inertia=i2)
    return b.build(gravity=gravity, name="double_pendulum")


def two_spheres(r1=0.05, r2=0.04, m1=1.0, m2=0.5, gap=-0.002, vel1=(0.3, 0.05, 0),
                vel2=(-0.2, 0, 0.1), spin1=(0, 0, 5.0), spin2=(1.0, 0, 0), mu=(0.7, 0.003, 0.0003),
                condim=3, k_user=0.1, d_user=0.001, offset=(0.0, 0.01, 0.005), gravity=(0, 0, 0)):
    """Two free spheres about to collide; no static geometry, gravity off by default."""
    b = _Builder(1)
    s1 = b.body(JNT_FREE, mass=m1, inertia=(0.4 * m1 * r1 * r1,) * 3)
    b.geom(SPHERE, s1, size=(r1, 0, 0), friction=mu)
    s2 = b.body(JNT_FREE, mass=m2, inertia=(0.4 * m2 * r2 * r2,) * 3)
    b.geom(SPHERE, s2, size=(r2, 0, 0), friction=mu)
    s = b.build(condim=condim, k_user=k_user, d_user=d_user, gravity=gravity, name="two_spheres")
    d = r1 + r2 + gap
    off = np.array(offset, float)
    dirv = np.array([1.0, 0, 0]) * math.sqrt(max(d * d - off @ off, 0.0)) + off
    s["q0"][0, 0:7] = (0, 0, 0.5, 1, 0, 0, 0)
    s["q0"][0, 7:14] = (*(np.array([0, 0, 0.5]) + dirv), 1, 0, 0, 0)
    s["v0"][0, 0:6] = (*vel1, *spin1)
    s["v0"][0, 6:12] = (*vel2, *spin2)
    return s


def sphere_cluster(nsphere=6, seed=0, condim=3, gravity=(0, 0, 0), k_user=0.1, d_user=0.001,
                   spread=0.07, speed=0.5, spin=5.0, ncon_max=64):
    """Free spheres packed closely with random velocities and spins, no static geoms."""
    rng = np.random.default_rng([seed, 3])
    b = _Builder(1)
    rad = rng.uniform(0.02, 0.05, nsphere)
    mass = 1000.0 * 4 / 3 * np.pi * rad ** 3
    for i in range(nsphere):
        bi = b.body(JNT_FREE, mass=mass[i], inertia=(0.4 * mass[i] * rad[i] ** 2,) * 3)
        b.geom(SPHERE, bi, size=(rad[i], 0, 0),
               friction=(rng.uniform(0.3, 1.0), rng.uniform(0.001, 0.005),
                         rng.uniform(0.0001, 0.0005)))
    s = b.build(condim=condim, k_user=k_user, d_user=d_user, gravity=gravity,
                ncon_max=ncon_max, name="sphere_cluster")
    q = s["q0"].reshape(nsphere, 7)
    q[:, 0:3] = rng.uniform(-spread, spread, (nsphere, 3))
    q[:, 3:7] = [_random_quat(rng) for _ in range(nsphere)]
    v = s["v0"].reshape(nsphere, 6)
    v[:, 0:3] = rng.normal(0, speed, (nsphere, 3))
    v[:, 3:6] = rng.normal(0, spin, (nsphere, 3))
    return s


def mixed_shapes(nworld=4, seed=0, condim=3, k_user=0.1, d_user=0.001, ncon_max=128):
    """Spheres, capsules and boxes over a tilted ground, a wall and a static sphere.

    Per-world random poses, sizes, masses and velocities; exercises every pair
    rule (plane-sphere, plane-capsule, plane-box, sphere-sphere, static sphere).
    """
    rng = np.random.default_rng([seed, 4])
    b = _Builder(nworld)
    b.geom(PLANE, -1, quat=_quat_z_to((0.05, -0.03, 1.0)))
    b.geom(PLANE, -1, pos=(0.3, 0, 0), quat=_quat_z_to((-1, 0, 0.1)), friction=(0.2, 0.001, 0))
    b.geom(SPHERE, -1, size=np.stack([rng.uniform(0.04, 0.06, nworld),
                                      np.zeros(nworld), np.zeros(nworld)], 1),
           pos=(-0.2, 0.1, 0.0))
    kinds = [SPHERE, CAPSULE, BOX, SPHERE, BOX, CAPSULE, SPHERE, SPHERE]
    nb = len(kinds)
    sizes = np.zeros((nworld, nb, 3))
    masses = np.zeros((nworld, nb))
    inert = np.zeros((nworld, nb, 3))
    for i, k in enumerate(kinds):
        if k == SPHERE:
            r = rng.uniform(0.02, 0.05, nworld)
            sizes[:, i, 0] = r
            masses[:, i] = 1000 * 4 / 3 * np.pi * r ** 3
            inert[:, i, :] = (0.4 * masses[:, i] * r * r)[:, None]
        elif k == CAPSULE:
            r = rng.uniform(0.015, 0.03, nworld)
            hl = rng.uniform(0.02, 0.05, nworld)
            sizes[:, i, 0], sizes[:, i, 1] = r, hl
            masses[:, i] = rng.uniform(0.1, 0.4, nworld)
            inert[:, i, 0] = inert[:, i, 1] = masses[:, i] * (3 * r * r + 4 * hl * hl) / 12
            inert[:, i, 2] = 0.5 * masses[:, i] * r * r
        else:
            hs = rng.uniform(0.02, 0.05, (nworld, 3))
            sizes[:, i] = hs
            masses[:, i] = rng.uniform(0.2, 1.0, nworld)
            inert[:, i, 0] = masses[:, i] * (hs[:, 1] ** 2 + hs[:, 2] ** 2) / 3
            inert[:, i, 1] = masses[:, i] * (hs[:, 0] ** 2 + hs[:, 2] ** 2) / 3
            inert[:, i, 2] = masses[:, i] * (hs[:, 0] ** 2 + hs[:, 1] ** 2) / 3
    for i, k in enumerate(kinds):
        bi = b.body(JNT_FREE, mass=masses[:, i], inertia=inert[:, i])
        fr = np.stack([rng.uniform(0.3, 1.0, nworld), rng.uniform(0.001, 0.005, nworld),
                       rng.uniform(0.0001, 0.0005, nworld)], 1)
        b.geom(k, bi, size=sizes[:, i], friction=fr)
    s = b.build(condim=condim, k_user=k_user, d_user=d_user, ncon_max=ncon_max,
                name="mixed_shapes")
    # bounding radius of each body; bodies start at most 1 cm into the ground
    bound = np.where(np.array(kinds) == SPHERE, sizes[:, :, 0],
                     np.where(np.array(kinds) == CAPSULE, sizes[:, :, 0] + sizes[:, :, 1],
                              np.linalg.norm(sizes, axis=2)))
    for w in range(nworld):
        q = s["q0"][w].reshape(nb, 7)
        v = s["v0"][w].reshape(nb, 6)
        for i in range(nb):
            q[i, 0:3] = (rng.uniform(-0.22, 0.22), rng.uniform(-0.15, 0.15),
                         bound[w, i] + rng.uniform(-0.01, 0.08))
            q[i, 3:7] = _random_quat(rng)
            v[i, 0:3] = rng.normal(0, 0.3, 3)
            v[i, 3:6] = rng.normal(0, 2.0, 3)
    return s


def pusher_ball(nworld=4, seed=0, condim=6, k_user=0.1, d_user=0.001, ncon_max=32):
    """A 3 cm free ball on the ground with four actuated 1 cm free spheres
    (fingertips driven by applied forces) pressed against it from four sides: a
    free-body stand-in for in-hand manipulation with the pair rules of the
    narrow phase (plane-sphere, sphere-sphere).  Per-world friction and pose
    jitter.  The ball's dofs are 0..5; fingertip f's force dofs are 6 + 6 f ..
    8 + 6 f."""
    rng = np.random.default_rng([seed, 6])
    b = _Builder(nworld)
    b.geom(PLANE, -1, friction=np.stack([rng.uniform(0.5, 0.9, nworld),
                                         np.full(nworld, 0.002), np.full(nworld, 0.0002)], 1))
    rb, mb = 0.03, 0.1
    ball = b.body(JNT_FREE, mass=mb, inertia=(0.4 * mb * rb * rb,) * 3)
    b.geom(SPHERE, ball, size=(rb, 0, 0),
           friction=np.stack([rng.uniform(0.4, 0.8, nworld), np.full(nworld, 0.002),
                              np.full(nworld, 0.0002)], 1))
    rf, mf = 0.01, 0.02
    for _ in range(4):
        t = b.body(JNT_FREE, mass=mf, inertia=(0.4 * mf * rf * rf,) * 3)
        b.geom(SPHERE, t, size=(rf, 0, 0),
               friction=np.stack([rng.uniform(0.6, 1.0, nworld), np.full(nworld, 0.002),
                                  np.full(nworld, 0.0002)], 1))
    s = b.build(condim=condim, k_user=k_user, d_user=d_user, ncon_max=ncon_max, name="pusher_ball")
    for w in range(nworld):
        q = s["q0"][w].reshape(5, 7)
        c = np.array([rng.uniform(-0.005, 0.005), rng.uniform(-0.005, 0.005), rb - 0.0005])
        q[0, 0:3] = c
        q[0, 3:7] = _random_quat(rng)
        for i in range(4):
            ang = 0.5 * np.pi * i + rng.uniform(-0.2, 0.2)
            el = rng.uniform(0.1, 0.4)  # elevation of the fingertip above the ball's equator
            d = np.array([np.cos(ang) * np.cos(el), np.sin(ang) * np.cos(el), np.sin(el)])
            q[1 + i, 0:3] = c + (rb + rf - 0.0005) * d
            q[1 + i, 3:7] = _random_quat(rng)
    return s


def select_worlds(scene, idx):
    """A copy of the scene restricted to the worlds in idx (any int sequence)."""
    idx = np.asarray(idx, np.int64)
    out = dict(scene)
    out["nworld"] = int(len(idx))
    for k in ("body_mass", "body_inertia", "geom_size", "geom_pos", "geom_quat",
              "geom_friction", "q0", "v0"):
        out[k] = np.ascontiguousarray(scene[k][idx])
    return out


def with_params(scene, **kw):
    """A shallow copy with scalar parameters replaced (h, k_user, d_user, margin, ...)."""
    out = dict(scene)
    for k, v in kw.items():
        if k in ("h", "k_user", "d_user", "margin"):
            out[k] = float(f32(v))
        elif k in ("gravity", "solimp"):
            out[k] = f32(np.asarray(v, float))
        else:
            out[k] = v
    return out


def articulated_mix(nworld=4, seed=0, condim=3, k_user=0.1, d_user=0.001, ncon_max=96):
    """Articulated bodies in contact: a 3-link hinge arm hanging from the world
    (capsule links, tip sphere), a slide-slide-hinge chain carrying a box, a
    floating base (free box with two hinged capsule fingers) and three free
    spheres, over a ground plane.  Per-world masses and random joint states."""
    rng = np.random.default_rng([seed, 5])
    b = _Builder(nworld)
    b.geom(PLANE, -1)
    cap_q = _quat_z_to((1.0, 0.0, 0.0))  # capsule axis along the link (+x)

    def m_(lo, hi):
        return rng.uniform(lo, hi, nworld)

    def inert(m, a, c):
        return np.stack([m * a, m * c, m * c], 1)

    # hinge arm from the world at (0.25, 0, 0.2), links along x
    parent = -1
    for i in range(3):
        L = 0.09
        m = m_(0.1, 0.3)
        bi = b.body(JNT_HINGE, parent, pos=(0.25, 0.0, 0.2) if i == 0 else (L, 0, 0),
                    axis=(0, 1, 0), ipos=(L / 2, 0, 0), mass=m, inertia=inert(m, 2e-4, 1e-3))
        b.geom(CAPSULE, bi, size=(0.015, L / 2 - 0.005, 0), pos=(L / 2, 0, 0), quat=cap_q,
               friction=(0.6, 0.003, 0.0003))
        parent = bi
    b.geom(SPHERE, parent, size=(0.025, 0, 0), pos=(0.09, 0, 0), friction=(0.8, 0.003, 0.0003))
    # slide x -> slide z -> hinge y carrying a box
    s0 = b.body(JNT_SLIDE, -1, pos=(-0.2, 0.2, 0.0), axis=(1, 0, 0), mass=0.05, inertia=(1e-5,) * 3)
    s1 = b.body(JNT_SLIDE, s0, axis=(0, 0, 1), mass=0.05, inertia=(1e-5,) * 3)
    mb = m_(0.3, 0.6)
    s2 = b.body(JNT_HINGE, s1, axis=(0, 1, 0), mass=mb, inertia=inert(mb, 6e-4, 6e-4))
    b.geom(BOX, s2, size=(0.04, 0.03, 0.025), friction=(0.5, 0.002, 0.0002))
    # floating base with two hinged fingers
    mp = m_(0.3, 0.5)
    fb = b.body(JNT_FREE, -1, pos=(-0.15, -0.15, 0.2), mass=mp, inertia=inert(mp, 1e-3, 1e-3))
    b.geom(BOX, fb, size=(0.05, 0.04, 0.015), friction=(0.7, 0.002, 0.0002))
    for sgn in (-1, 1):
        mf = m_(0.05, 0.1)
        fi = b.body(JNT_HINGE, fb, pos=(0.05, 0.025 * sgn, 0.0), axis=(0, 1, 0), ipos=(0.03, 0, 0),
                    mass=mf, inertia=inert(mf, 1e-5, 5e-5))
        b.geom(CAPSULE, fi, size=(0.01, 0.025, 0), pos=(0.03, 0, 0), quat=cap_q,
               friction=(0.9, 0.003, 0.0003))
    # free spheres
    for _ in range(3):
        r = rng.uniform(0.02, 0.035, nworld)
        m = 1000 * 4 / 3 * np.pi * r ** 3
        bi = b.body(JNT_FREE, mass=m, inertia=np.repeat((0.4 * m * r * r)[:, None], 3, 1))
        b.geom(SPHERE, bi, size=np.stack([r, 0 * r, 0 * r], 1), friction=(0.6, 0.003, 0.0003))
    s = b.build(condim=condim, k_user=k_user, d_user=d_user, ncon_max=ncon_max,
                name="articulated_mix")
    qa = qadr(s)
    da = dadr(s)
    for w in range(nworld):
        q, v = s["q0"][w], s["v0"][w]
        for i in range(3):                       # arm angles
            q[qa[i]] = rng.uniform(-0.4, 1.2)
            v[da[i]] = rng.normal(0, 1.0)
        q[qa[3]], q[qa[4]], q[qa[5]] = rng.uniform(-0.05, 0.05), rng.uniform(0.03, 0.08), rng.uniform(-0.5, 0.5)
        v[da[3]], v[da[4]], v[da[5]] = rng.normal(0, 0.2), rng.normal(0, 0.2), rng.normal(0, 1.0)
        q[qa[6]:qa[6] + 3] = (-0.15 + rng.uniform(-0.03, 0.03), -0.15 + rng.uniform(-0.03, 0.03),
                              rng.uniform(0.05, 0.12))
        q[qa[6] + 3:qa[6] + 7] = _random_quat(rng) * 0.2 + np.array([1.0, 0, 0, 0])
        q[qa[6] + 3:qa[6] + 7] /= np.linalg.norm(q[qa[6] + 3:qa[6] + 7])
        v[da[6]:da[6] + 6] = rng.normal(0, 0.3, 6)
        q[qa[7]], q[qa[8]] = rng.uniform(-0.5, 0.5), rng.uniform(-0.5, 0.5)
        for i in range(3):
            bi = 9 + i
            q[qa[bi]:qa[bi] + 3] = (rng.uniform(-0.25, 0.3), rng.uniform(-0.2, 0.2), rng.uniform(0.03, 0.25))
            q[qa[bi] + 3:qa[bi] + 7] = (1, 0, 0, 0)
            v[da[bi]:da[bi] + 3] = rng.normal(0, 0.3, 3)
    return s


# Synthetic four-finger hand (16 hinge dofs) around a free 5 cm cube.
HAND_LINKS = (0.02, 0.04, 0.03, 0.025)     # base (abduction), proximal, middle, distal [m]
# Position gains per finger joint: omega^2 I and 2 zeta omega I with omega = 120 rad/s,
# zeta = 0.5 and I the joint's effective inertia at the rest pose (1 / (M^-1)_jj), which
# keeps h^2 eig(M^-1 Kp) and h eig(M^-1 Kd) at about 0.14 and 0.6 for h = 2 ms.
HAND_KP = (10.71, 1.509, 0.1875, 0.0511)   # [N m / rad]
HAND_KD = (0.0893, 0.01257, 0.00156, 0.000426)  # [N m s / rad]
HAND_Q0 = (0.0, -0.5, 0.8, 0.7)            # rest pose: fingertips 4.2 cm from the cube's axis [rad]


def hand_cube(nworld=4, seed=0, condim=6, k_user=0.1, d_user=0.002, h=0.002, ncon_max=64):
    """Four fingers of four hinges each (abduction about the root's z, then
    three flexion hinges about y; capsule links, fingertip spheres), rooted on
    a palm plane around a free 5 cm cube (body 0) resting on it; position
    actuators on the 16 finger dofs (gains HAND_KP, HAND_KD; the step input of
    a finger dof is its target angle).  nv = 22.  Per world the cube's yaw and
    position and the fingers' angles are perturbed (seeded)."""
    rng = np.random.default_rng([seed, 11])
    b = _Builder(nworld)
    b.geom(PLANE, -1, friction=(0.6, 0.005, 0.0002))
    half = 0.025
    mc = 0.1
    ic = mc * (2 * half) ** 2 / 6
    cube = b.body(JNT_FREE, pos=(0, 0, half), mass=mc, inertia=(ic, ic, ic))
    b.geom(BOX, cube, size=(half, half, half), friction=(0.8, 0.005, 0.0002))
    cap_q = _quat_z_to((1.0, 0.0, 0.0))  # capsule axis along the link (+x)
    r_link, r_tip, m_link = 0.01, 0.011, 0.05
    for f in range(4):
        psi = f * math.pi / 2                          # azimuth of the finger root (facing a cube face)
        root = (0.139 * math.cos(psi), 0.139 * math.sin(psi), 0.03)
        yaw = psi + math.pi                            # local +x toward the cube
        parent = -1
        for j, L in enumerate(HAND_LINKS):
            ixx = 0.5 * m_link * r_link ** 2
            iyy = m_link * (L * L / 12 + r_link ** 2 / 4)
            kw = dict(axis=(0, 0, 1) if j == 0 else (0, 1, 0), ipos=(L / 2, 0, 0), mass=m_link,
                      inertia=(ixx, iyy, iyy))
            if j == 0:
                bi = b.body(JNT_HINGE, -1, pos=root, quat=(math.cos(yaw / 2), 0, 0, math.sin(yaw / 2)), **kw)
            else:
                bi = b.body(JNT_HINGE, parent, pos=(HAND_LINKS[j - 1], 0, 0), **kw)
            b.geom(CAPSULE, bi, size=(r_link, L / 2, 0), pos=(L / 2, 0, 0), quat=cap_q,
                   friction=(1.0, 0.005, 0.0002))
            parent = bi
        b.geom(SPHERE, parent, size=(r_tip, 0, 0), pos=(HAND_LINKS[-1], 0, 0), friction=(1.0, 0.005, 0.0002))
    s = b.build(condim=condim, k_user=k_user, d_user=d_user, h=h, ncon_max=ncon_max, name="hand_cube")
    nv = dims(s)[1]
    kp, kd = np.zeros(nv), np.zeros(nv)
    kp[6:] = np.tile(HAND_KP, 4)
    kd[6:] = np.tile(HAND_KD, 4)
    s["dof_kp"], s["dof_kd"] = f32(kp), f32(kd)
    for w in range(nworld):
        q = s["q0"][w]
        a = rng.uniform(-0.1, 0.1)
        q[0:3] = (rng.uniform(-0.005, 0.005), rng.uniform(-0.005, 0.005), half + 0.001)
        q[3:7] = (math.cos(a / 2), 0, 0, math.sin(a / 2))
        q[7:] = np.tile(HAND_Q0, 4) + rng.uniform(-0.03, 0.03, 16)
    return s


def hand_targets(scene):
    """[nworld][nv] step input holding every finger at its initial angle (the
    cube's dofs take zero force)."""
    tau = np.zeros((scene["nworld"], dims(scene)[1]), np.float32)
    tau[:, 6:] = scene["q0"][:, 7:]
    return tau

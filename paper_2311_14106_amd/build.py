"""Build libmdmrg.so in-tree for gfx950 with hipcc, and the range-checking
host-only variant libmdmrg_check.so (device layer replaced by
csrc/device_check.cpp: no GPU, no arithmetic, every device access checked).

Usage: python -m paper_2311_14106_amd.build [--check]   (or build() / build_check())
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, 'csrc')
OUT = os.path.join(HERE, 'libmdmrg.so')
HIPCC = os.environ.get('HIPCC', '/opt/rocm/bin/hipcc')
CXX = os.environ.get('CXX', 'g++')

SOURCES = ['device.hip', 'model.cpp', 'engine.cpp', 'capi.cpp', 'modes.cpp']
COMMON = ['-O3', '-fPIC', '-std=c++17', '-Wall', '-Wno-unused-result', '-pthread']
HIP_FLAGS = ['-x', 'hip', '--offload-arch=gfx950',
             '-Xclang', '-target-feature', '-Xclang', '-packed-fp32-ops']


def build(verbose=False):
    objdir = os.path.join(HERE, '_build')
    os.makedirs(objdir, exist_ok=True)
    objs = []
    for src in SOURCES:
        path = os.path.join(CSRC, src)
        obj = os.path.join(objdir, src + '.o')
        if src.endswith('.hip'):
            cmd = [HIPCC] + COMMON + HIP_FLAGS
        else:
            cmd = [CXX] + COMMON
        cmd += ['-I', os.path.join(HERE, '..', 'include'), '-c', path, '-o', obj]
        if verbose:
            print(' '.join(cmd), flush=True)
        subprocess.check_call(cmd)
        objs.append(obj)
    tmp = OUT + '.tmp'
    cmd = [HIPCC, '-shared', '-fPIC', '--offload-arch=gfx950', '-o', tmp] + objs + \
          ['-L/opt/rocm/lib', '-lrocsolver', '-lrocblas', '-pthread', '-Wl,-rpath,/opt/rocm/lib']
    if verbose:
        print(' '.join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, OUT)
    return OUT


CHECK_OUT = os.path.join(HERE, 'libmdmrg_check.so')
CHECK_SOURCES = ['device_check.cpp', 'model.cpp', 'engine.cpp', 'capi.cpp', 'modes.cpp']


def build_check(verbose=False):
    """Host-only build with the range-checking device layer (g++, -O2)."""
    objdir = os.path.join(HERE, '_build', 'check')
    os.makedirs(objdir, exist_ok=True)
    objs = []
    for src in CHECK_SOURCES:
        obj = os.path.join(objdir, src + '.o')
        cmd = [CXX, '-O2', '-fPIC', '-std=c++17', '-Wall', '-Wno-unused-result', '-pthread',
               '-I', os.path.join(HERE, '..', 'include'), '-c', os.path.join(CSRC, src), '-o', obj]
        if verbose:
            print(' '.join(cmd), flush=True)
        subprocess.check_call(cmd)
        objs.append(obj)
    tmp = CHECK_OUT + '.tmp'
    cmd = [CXX, '-shared', '-fPIC', '-pthread', '-o', tmp] + objs
    subprocess.check_call(cmd)
    os.replace(tmp, CHECK_OUT)
    return CHECK_OUT


if __name__ == '__main__':
    if '--check' in sys.argv:
        print(build_check(verbose='-v' in sys.argv))
    else:
        print(build(verbose='-v' in sys.argv))

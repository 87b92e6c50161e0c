"""Wire format of the streaming sample application (CPU only): messages
round-trip over a socket pair, the end marker ends the stream, and a stream
cut inside a message or with a wrong magic is refused."""
import socket
import struct

import pytest

from paper_2208_01641_amd import stream


def test_messages_round_trip_and_end_marker():
    a, b = socket.socketpair()
    msgs = [(0, 123, b""), (1, 2 ** 40, bytes(range(256)) * 40), (7, 5, b"\x00" * 3)]
    for i, t, p in msgs:
        a.sendall(stream.pack_message(i, t, p))
    a.sendall(stream.HEADER.pack(stream.MAGIC, stream.END, 0, 0))
    for m in msgs:
        assert stream.read_message(b) == m
    assert stream.read_message(b) is None
    a.close()
    b.close()


def test_truncated_and_foreign_streams_are_refused():
    a, b = socket.socketpair()
    a.sendall(stream.pack_message(3, 9, b"abcdef")[:-2])
    a.close()
    with pytest.raises(ConnectionError):
        stream.read_message(b)
    b.close()
    a, b = socket.socketpair()
    a.sendall(struct.pack("<4sIQI", b"XXXX", 0, 0, 0))
    with pytest.raises(ValueError):
        stream.read_message(b)
    a.close()
    b.close()
